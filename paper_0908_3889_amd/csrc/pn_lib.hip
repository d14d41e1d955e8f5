// pn_lib.hip -- gfx950 kernels and the C interface declared in include/pn.h.
//
// The hot path: one inspiral per lane, its state, stage vectors and
// coefficient row in registers; adaptive Dormand-Prince RK5(4) with FSAL
// (Sec. II: Dormand-Prince, tolerance, h = 10); termination at omega_f by a
// last stretch integrated with omega as the independent variable; a
// persistent grid in which a wave hands new inspirals to its idle lanes
// (ballot + one atomic add per wave) so that inspirals of very different
// lengths share lanes without leaving them idle.
//
// Two precisions share the scheduling code through a policy:
//   F64       everything in FP64;
//   F32Split  stages, right-hand sides, increments and error estimate in
//             FP32; the state, t, h, the error norm, the step control and
//             the omega >= omega_f test in FP64 (each FP32 increment is added
//             to the FP64 state, so rounding does not build up in the state).
#include <hip/hip_runtime.h>

#include <atomic>
#include <cstring>
#include <mutex>

#include "pn.h"
#include "pn_adjoint.hpp"
#include "pn_device.hpp"
#include "pn_slots.hpp"

namespace pn {

// Occupancy targets (waves per SIMD) the integration kernels are compiled
// for; chosen by measurement (register budget 512/target per lane).
constexpr int kWpeF64 = 2;
constexpr int kWpeF32 = 3;     // FP32-split
constexpr int kWpeF32S = 3;    // FP32-state (4 spills 23 VGPRs and is slower)

// ---------------------------------------------------------------------------
// Dormand-Prince RK5(4)7M tableau (Dormand & Prince 1980)
// ---------------------------------------------------------------------------
constexpr double A21 = 1.0 / 5.0;
constexpr double A31 = 3.0 / 40.0, A32 = 9.0 / 40.0;
constexpr double A41 = 44.0 / 45.0, A42 = -56.0 / 15.0, A43 = 32.0 / 9.0;
constexpr double A51 = 19372.0 / 6561.0, A52 = -25360.0 / 2187.0, A53 = 64448.0 / 6561.0,
                 A54 = -212.0 / 729.0;
constexpr double A61 = 9017.0 / 3168.0, A62 = -355.0 / 33.0, A63 = 46732.0 / 5247.0,
                 A64 = 49.0 / 176.0, A65 = -5103.0 / 18656.0;
// 5th-order weights (= stage-7 row, FSAL); b2 = b7 = 0
constexpr double B1 = 35.0 / 384.0, B3 = 500.0 / 1113.0, B4 = 125.0 / 192.0,
                 B5 = -2187.0 / 6784.0, B6 = 11.0 / 84.0;
// error weights e = b - bhat; e2 = 0
constexpr double E1 = 71.0 / 57600.0, E3 = -71.0 / 16695.0, E4 = 71.0 / 1920.0,
                 E5 = -17253.0 / 339200.0, E6 = 22.0 / 525.0, E7 = -1.0 / 40.0;

// accept when err = sqrt(z) <= 1, i.e. z <= 1 + 2^-52 (sqrt rounds that to 1)
constexpr double Z_ACCEPT = 1.0 + 2.220446049250313e-16;

struct Uni {
    double omega_f, tol, h0, h_fixed, t_end;
    TermConsts tc;
    TermConstsF tcf;
    int64_t n, ld, max_steps;
    int terms, theta_literal;
    int fixed, tend;
    int refill_min;
    int rr_on;
    // tape for the adjoint: per inspiral, [n_t, n_w, h_0 .. h_{cap-1},
    // checkpoints y(step jK), j = 0 .. cap/K] (doubles, `tape_stride` apart)
    double* tape;
    int64_t tape_stride;
    int tape_cap, ckpt_every;
};

struct Io {
    const double* __restrict__ m;
    const double* __restrict__ S0;
    const double* __restrict__ L0;
    const double* __restrict__ w0;
    double* __restrict__ y;
    double* __restrict__ t;
    int32_t* __restrict__ steps;
    int32_t* __restrict__ status;
    double* __restrict__ dots;
    double* __restrict__ phase;   // orbital phase at t_final, or null
    const int32_t* __restrict__ order;   // hand-out order of the inspirals, or null
    const double* __restrict__ packed;   // inputs as [n][16] records, or null
};

// What a persistent launch reads only when it refills lanes or writes
// outputs; kept in device memory (the call's slot) instead of kernel
// arguments, so that these values do not occupy scalar registers in the
// step loop.
struct LaunchDesc {
    Io io;
    Uni u;
};
constexpr int kDescOffset = 32;   // words: the counter, then padding to 256 B (its own cache lines)
constexpr int kSlotWords = 64;    // 512 B per call slot
static_assert(sizeof(LaunchDesc) / 8 + kDescOffset <= kSlotWords, "launch descriptor does not fit its slot");
static_assert(sizeof(LaunchDesc) % 8 == 0 && sizeof(LaunchDesc) / 8 <= 64, "descriptor copy uses one word per thread");

__device__ __forceinline__ bool finite(double v) { return __builtin_isfinite(v); }

// An empty asm that takes v in a register: the accumulation that produced v is
// completed here instead of being deferred (with its operands kept alive).
__device__ __forceinline__ void settle(double& v) { __asm__ volatile("" : "+v"(v)); }
__device__ __forceinline__ void settle(float& v) { __asm__ volatile("" : "+v"(v)); }

template <bool PHASE = false>
__device__ void write_out(const Io& io, const Uni& u, int64_t i, const double* y, double t, int acc,
                          int rej, int nrhs, int st, double phase = 0.0) {
    const int64_t ld = u.ld;
#pragma unroll
    for (int c = 0; c < 10; ++c) io.y[c * ld + i] = y[c];
    io.t[i] = t;
    if (PHASE) io.phase[i] = phase;
    io.steps[i] = acc;
    io.steps[ld + i] = rej;
    io.steps[2 * ld + i] = nrhs;
    io.status[i] = st;
    if (io.dots) {
        const double n1 = __builtin_sqrt(y[1] * y[1] + y[2] * y[2] + y[3] * y[3]);
        const double n2 = __builtin_sqrt(y[4] * y[4] + y[5] * y[5] + y[6] * y[6]);
        const double nl = __builtin_sqrt(y[7] * y[7] + y[8] * y[8] + y[9] * y[9]);
        const double s12 = y[1] * y[4] + y[2] * y[5] + y[3] * y[6];
        const double s1l = y[1] * y[7] + y[2] * y[8] + y[3] * y[9];
        const double s2l = y[4] * y[7] + y[5] * y[8] + y[6] * y[9];
        io.dots[i] = (n1 > 0.0 && n2 > 0.0) ? s12 / (n1 * n2) : 0.0;
        io.dots[ld + i] = (n1 > 0.0 && nl > 0.0) ? s1l / (n1 * nl) : 0.0;
        io.dots[2 * ld + i] = (n2 > 0.0 && nl > 0.0) ? s2l / (n2 * nl) : 0.0;
    }
}

// Read inspiral idx into y and the masses; returns 0, or the status of an
// inspiral that is finished at once (bad input, or omega0 >= omega_f), whose
// outputs are then already written.  From the packed record when there is
// one (six 16-byte loads from one cache line), else from the SoA inputs.
template <bool PHASE = false>
__device__ int read_input(const Io& io, const Uni& u, int64_t idx, double* y, double& m1, double& m2) {
    const int64_t ld = u.ld;
    if (io.packed) {
        const double2* r = (const double2*)(io.packed + idx * 16);
        const double2 a = r[0], b = r[1], c = r[2], d = r[3], e = r[4], f = r[5];
        m1 = a.x; m2 = a.y;
        y[0] = b.x; y[1] = b.y; y[2] = c.x; y[3] = c.y; y[4] = d.x;
        y[5] = d.y; y[6] = e.x; y[7] = e.y; y[8] = f.x; y[9] = f.y;
    } else {
        m1 = io.m[idx];
        m2 = io.m[ld + idx];
        y[0] = io.w0[idx];
#pragma unroll
        for (int c = 0; c < 6; ++c) y[1 + c] = io.S0[c * ld + idx];
#pragma unroll
        for (int c = 0; c < 3; ++c) y[7 + c] = io.L0[c * ld + idx];
    }
    bool bad = !(m1 > 0.0) || !(m2 > 0.0) || !(y[0] > 0.0) || !finite(m1) || !finite(m2);
#pragma unroll
    for (int c = 0; c < 10; ++c) bad = bad || !finite(y[c]);
    if (bad) { write_out<PHASE>(io, u, idx, y, 0.0, 0, 0, 0, PN_ST_BAD_INPUT); return PN_ST_BAD_INPUT; }
    if (!u.tend && !(y[0] < u.omega_f)) {
        write_out<PHASE>(io, u, idx, y, 0.0, 0, 0, 0, PN_ST_DONE_AT_START);
        return PN_ST_DONE_AT_START;
    }
    return 0;
}

// mean_c (e_c / sc_c)^2 with sc_c = tol + tol max(|y_c|, |ynew_c|): the squared
// RMS error norm z = err^2 of the error estimate e (the FP64 stepper passes
// e/h and scales the result by h^2).  One reciprocal per component: the
// FP32-state stepper (the grouped forms below fall back to the same sum).
__device__ __forceinline__ double error_norm_each(const Uni& u, const double* y, const double* ynew, const double* e) {
    double z = 0.0;
#pragma unroll
    for (int c = 0; c < 10; ++c) {
        const double sc = __builtin_fma(u.tol, fmax_abs(y[c], ynew[c]), u.tol);
        const double q = e[c] * rcp_1step(sc);
        z = __builtin_fma(q, q, z);
    }
    return z * 0.1;
}

// The same norm with the reciprocals taken in pairs (1/s0 = s1 / (s0 s1)):
// the FP32-split stepper, where it saves 2 % of the kernel time without
// spilling at 3 waves per SIMD (the FP32-state stepper measured no gain).
// Lanes with a pair product outside the normal range take one reciprocal per
// component.
__device__ __forceinline__ double error_norm_pairs(const Uni& u, const double* y, const double* ynew, const double* e) {
    double z = 0.0;
    bool bad = false;
#pragma unroll
    for (int c = 0; c < 10; c += 2) {
        const double s0 = __builtin_fma(u.tol, fmax_abs(y[c], ynew[c]), u.tol);
        const double s1 = __builtin_fma(u.tol, fmax_abs(y[c + 1], ynew[c + 1]), u.tol);
        const double p = s0 * s1;
        bad = bad || __builtin_amdgcn_class(p, 0x2ff);   // every class but +normal
        const double r = rcp_1step(p);
        const double q0 = e[c] * (r * s1), q1 = e[c + 1] * (r * s0);
        z = __builtin_fma(q0, q0, z);
        z = __builtin_fma(q1, q1, z);
    }
    if (__builtin_expect(__ballot(bad) != 0, 0)) {
        if (bad) {
            z = 0.0;
#pragma unroll
            for (int c = 0; c < 10; ++c) {
                const double q = e[c] * rcp_1step(__builtin_fma(u.tol, fmax_abs(y[c], ynew[c]), u.tol));
                z = __builtin_fma(q, q, z);
            }
        }
    }
    return z * 0.1;
}

// 1/s0 .. 1/s3 from the reciprocal of their product (1/s0 = s1 s2 s3 / (s0 s1
// s2 s3), and so on); bad is set when the product is not a positive normal
// number, where that reciprocal cannot be trusted.
__device__ __forceinline__ void rcp4(double s0, double s1, double s2, double s3, double& i0, double& i1,
                                     double& i2, double& i3, bool& bad) {
    const double p01 = s0 * s1, p23 = s2 * s3;
    const double P = p01 * p23;
    bad = bad || __builtin_amdgcn_class(P, 0x2ff);   // every class but +normal
    const double r = rcp_1step(P);
    const double r01 = r * p23, r23 = r * p01;
    i0 = r01 * s1; i1 = r01 * s0; i2 = r23 * s3; i3 = r23 * s2;
}

// The same norm (FP64 stepper) with the ten reciprocals taken in groups of
// four, four and two.  FP64 reciprocals issue at a quarter of the FMA rate:
// three of them and 15 multiplications cost less than ten, and the result
// differs from one reciprocal per component by a few ulp.  Lanes with a group
// product outside the normal range (tolerances or states far beyond double
// precision) take one reciprocal per component instead.
__device__ __forceinline__ double error_norm(const Uni& u, const double* y, const double* ynew, const double* e) {
    double sc[10], iv[10];
#pragma unroll
    for (int c = 0; c < 10; ++c) sc[c] = __builtin_fma(u.tol, fmax_abs(y[c], ynew[c]), u.tol);
    bool bad = false;
    rcp4(sc[0], sc[1], sc[2], sc[3], iv[0], iv[1], iv[2], iv[3], bad);
    rcp4(sc[4], sc[5], sc[6], sc[7], iv[4], iv[5], iv[6], iv[7], bad);
    {
        const double p = sc[8] * sc[9];
        bad = bad || __builtin_amdgcn_class(p, 0x2ff);
        const double r = rcp_1step(p);
        iv[8] = r * sc[9];
        iv[9] = r * sc[8];
    }
    double z = 0.0;
#pragma unroll
    for (int c = 0; c < 10; ++c) {
        const double q = e[c] * iv[c];
        z = __builtin_fma(q, q, z);
    }
    if (__builtin_expect(__ballot(bad) != 0, 0)) {
        if (bad) {
            z = 0.0;
#pragma unroll
            for (int c = 0; c < 10; ++c) {
                const double q = e[c] * rcp_1step(sc[c]);
                z = __builtin_fma(q, q, z);
            }
        }
    }
    return z * 0.1;
}

// omega-mode: divide the RHS by omega-dot and put 1 in the omega slot.  One
// Newton step (about 11 ulp) suffices: the scaled derivatives only enter
// the state through increments far smaller than the state itself.
__device__ __forceinline__ double recip(double d) { return rcp_1step(d); }
__device__ __forceinline__ float recip(float d) { return __builtin_amdgcn_rcpf(d); }

template <class T>
__device__ __forceinline__ void to_omega_variable(T* k, T& dt, bool om) {
    const T s = om ? recip(k[0]) : T(1);
#pragma unroll
    for (int c = 1; c < 10; ++c) k[c] *= s;
    k[0] = om ? T(1) : k[0];
    dt = s;
}

__device__ __forceinline__ double* tape_of(const Uni& u, int64_t idx) { return u.tape + idx * u.tape_stride; }

__device__ __forceinline__ void tape_checkpoint(const Uni& u, int64_t idx, int j, const double* y) {
    double* ck = tape_of(u, idx) + 2 + u.tape_cap + (int64_t)j * 10;
#pragma unroll
    for (int c = 0; c < 10; ++c) ck[c] = y[c];
}

// Outcome known before a step (in this order of precedence): the step limit,
// a full tape, d omega/dt <= 0.
template <bool RECORD, class LaneT>
__device__ __forceinline__ int pre_status(const Uni& u, const LaneT& L) {
    int st = 0;
    if (L.omega_mode ? L.dt1 <= 0 : (u.rr_on && L.k1[0] <= 0)) st = PN_ST_OMEGADOT_NONPOSITIVE;
    if (RECORD && L.acc >= u.tape_cap) st = PN_ST_TAPE_FULL;
    if (L.acc + L.rej >= u.max_steps) st = PN_ST_MAX_STEPS;
    return st;
}

// The step to attempt, clipped to what is left of the omega stretch (or of
// t_end); last = the clipped step ends the integration if accepted.
// GEN = false: the kernel only runs adaptive integrations to omega_f (no
// fixed step, no t_end), so those tests fold away.
template <bool GEN, class LaneT>
__device__ __forceinline__ double clip_step(const Uni& u, const LaneT& L, bool& last) {
    const double remain = L.omega_mode ? u.omega_f - L.omega() : (GEN ? u.t_end - L.t : 0.0);
    last = (L.omega_mode || (GEN && u.tend)) && L.h >= remain;
    return last ? remain : L.h;
}

// Acceptance test and state update of an attempted step of size h, applied
// on lanes with go = (active, no status before the step); other lanes keep
// their state.  Y: candidate state, k7/dt7: its derivative, dts = sum_j b_j
// dt_j (omega mode).  Returns 0 (continue), 1 (finished OK) or a status.
template <bool RECORD, bool GEN, class LaneT, class KT>
__device__ __forceinline__ int control(const Uni& u, LaneT& L, bool go, int st, bool fin, double z, double h,
                                       bool last, const double* Y, const KT* k7, KT dt7, KT dts) {
    const bool fixed = GEN && u.fixed, tend = GEN && u.tend;
    if (go && !fin) st = PN_ST_NONFINITE;
    const bool ok = go && fin;
    const bool acc = ok && (fixed || z <= Z_ACCEPT);
    // a candidate past omega_f is discarded: the stretch is finished with
    // omega as the independent variable
    const bool to_w = acc && !L.omega_mode && !tend && Y[0] > u.omega_f;
    const bool take = acc && !to_w;
    const bool rej = ok && !acc;
    // step factor (safety 0.9, exponent 1/5, clamped to [0.2, 5], no growth
    // right after a rejection); one z^(-1/10) serves accepts and rejects
    double fac = 1.0;
    if (!fixed) {
        const double p = pow_m_tenth_scaled(fmin_k(fmax_k(z, 9.313225746154785e-10), 1.073741824e9), 0.9);
        const double lo = fmax_k(p, 0.2);
        fac = rej ? lo : fmin_k(lo, L.last_rej ? 1.0 : 5.0);
    }
    // The state is updated with selects rather than a divergent branch, so
    // that y and k1 keep their registers across the loop.
    if (__builtin_expect(__ballot(to_w) != 0, 0)) {
        const KT s = to_w ? KT(1) / L.k1[0] : KT(1);
#pragma unroll
        for (int c = 1; c < 10; ++c) L.k1[c] *= s;
        L.k1[0] = to_w ? KT(1) : L.k1[0];
        L.dt1 = to_w ? s : L.dt1;
        L.nt = to_w ? L.acc : L.nt;
        L.h = to_w ? u.omega_f - L.omega() : L.h;
        L.last_rej = to_w ? false : L.last_rej;
        L.omega_mode = L.omega_mode || to_w;
    }
    if (RECORD && take) {
        tape_of(u, L.idx)[2 + L.acc] = h;
        if ((L.acc + 1) % u.ckpt_every == 0) tape_checkpoint(u, L.idx, (L.acc + 1) / u.ckpt_every, Y);
    }
    const double tn = L.omega_mode ? __builtin_fma(h, (double)dts, L.t) : L.t + h;
    const bool done = take && (last || (!L.omega_mode && !tend && Y[0] == u.omega_f));
    if (take) L.take(Y, k7);
    if (done && L.omega_mode) L.set_omega(u.omega_f);
    L.t = take ? tn : L.t;
    L.dt1 = take ? dt7 : L.dt1;
    L.acc += take ? 1 : 0;
    L.rej += rej ? 1 : 0;
    const bool resize = rej || (take && !done && !fixed);
    L.h = resize ? h * fac : L.h;
    L.last_rej = resize ? rej : L.last_rej;
    const double scale = L.omega_mode ? __builtin_fabs(L.omega()) : __builtin_fmax(1.0, __builtin_fabs(L.t));
    if (rej && L.h < 1e-14 * scale) st = PN_ST_H_UNDERFLOW;
    return st != 0 ? st : (done ? 1 : 0);
}

// ===========================================================================
// FP64 lane
// ===========================================================================
struct LaneF64 {
    double y[10];
    double k1[10];
    double lnv;       // ln|M omega| at y, carried from the stage that produced y
    double x;         // (M omega)^{1/3} at y, carried likewise
    double dt1;       // dt/d(variable) of k1: 1 in time mode, 1/omega-dot in omega mode
    double t, h;
    double phase;     // integral of omega dt (phase kernels only)
    Row row;
    int64_t idx;
    int acc, rej, nrhs;
    int nt;           // accepted time steps (recording only)
    bool omega_mode, last_rej;
    __device__ __forceinline__ double omega() const { return y[0]; }
    __device__ __forceinline__ void set_omega(double w) { y[0] = w; }
    // an accepted candidate state and its derivative
    __device__ __forceinline__ void take(const double* Y, const double* k) {
#pragma unroll
        for (int c = 0; c < 10; ++c) {
            y[c] = Y[c];
            k1[c] = k[c];
        }
    }
};

// PHASE: also integrate the orbital phase, d Phi/dt = omega, as a quadrature
// on the same steps (5th-order weights on the stage values of omega times
// dt/d(variable)), outside the error norm, so the steps are unchanged.
template <bool RECORD, bool PHASE = false, bool GEN = true>
struct F64 {
    using LaneT = LaneF64;

    static __device__ int load(const Io& io, const Uni& u, LaneT& L, int64_t idx) {
        L.idx = idx;
        double m1, m2;
        const int st = read_input<PHASE>(io, u, idx, L.y, m1, m2);
        if (st) return st;
        L.t = 0.0;
        L.acc = 0; L.rej = 0;
        L.omega_mode = false; L.last_rej = false;
        L.h = u.fixed ? u.h_fixed : u.h0;
        L.phase = 0.0;
        make_row(L.row, m1, m2, u.terms, u.theta_literal);
        LogBase lb;
        L.lnv = rhs_x<Row, false>(L.row, u.tc, lb, L.y, L.k1, L.x);
        L.dt1 = 1.0;
        L.nrhs = 1;
        L.nt = 0;
        if (RECORD) tape_checkpoint(u, idx, 0, L.y);
        return 0;
    }

    static __device__ void finish(const Io& io, const Uni& u, const LaneT& L, int st) {
        write_out<PHASE>(io, u, L.idx, L.y, L.t, L.acc, L.rej, L.nrhs, st, L.phase);
        if (RECORD) {
            double* tp = tape_of(u, L.idx);
            const int nt = L.omega_mode ? L.nt : L.acc;
            tp[0] = (double)nt;
            tp[1] = (double)(L.acc - nt);
        }
    }

    // One attempted step.  Every lane of the wave runs it; lanes that are not
    // active compute on their stale state and change nothing.  Returns 0 =
    // continue, 1 = finished OK, < 0 = status (meaningful on active lanes).
    static __device__ __forceinline__ int step(const Uni& u, LaneT& L, bool active, bool any_w) {
        const int st0 = pre_status<RECORD>(u, L);
        const bool go = active && st0 == 0;
        bool last;
        // idle lanes take a step of zero: their stage points stay on their
        // state, so they never send the wave down a slow path
        const double h = active ? clip_step<GEN>(u, L, last) : 0.0;

        const Row& R = L.row;
        const double* y = L.y;
        const double* k1 = L.k1;
        double Y[10], k2[10], k3[10], k4[10], k5[10], k6[10];
        double dtj;
        double dts = B1 * L.dt1;     // sum_j b_j dt_j, used in omega mode only
        double ps = 0.0;             // sum_j b_j omega_j dt_j (PHASE)
        if (PHASE) ps = B1 * (y[0] * L.dt1);
        LogBase lb;
        lb.w = y[0];
        lb.iw = rcp_1step(y[0]);     // only scales the small offset u of the stage points
        lb.lnv = L.lnv;
        lb.x = L.x;
        {
            const double c1 = h * A21;
#pragma unroll
            for (int c = 0; c < 10; ++c) Y[c] = __builtin_fma(c1, k1[c], y[c]);
            rhs<Row, true>(R, u.tc, lb, Y, k2);
            if (__builtin_expect(any_w, 0)) to_omega_variable(k2, dtj, L.omega_mode);
        }
        {
            const double c1 = h * A31, c2 = h * A32;
#pragma unroll
            for (int c = 0; c < 10; ++c) Y[c] = __builtin_fma(c2, k2[c], __builtin_fma(c1, k1[c], y[c]));
            rhs<Row, true>(R, u.tc, lb, Y, k3);
            if (__builtin_expect(any_w, 0)) { to_omega_variable(k3, dtj, L.omega_mode); dts = __builtin_fma(B3, dtj, dts); settle(dts); }
            if (PHASE) { ps = __builtin_fma(B3, Y[0] * (any_w ? dtj : 1.0), ps); settle(ps); }
        }
        {
            const double c1 = h * A41, c2 = h * A42, c3 = h * A43;
#pragma unroll
            for (int c = 0; c < 10; ++c)
                Y[c] = __builtin_fma(c3, k3[c], __builtin_fma(c2, k2[c], __builtin_fma(c1, k1[c], y[c])));
            rhs<Row, true>(R, u.tc, lb, Y, k4);
            if (__builtin_expect(any_w, 0)) { to_omega_variable(k4, dtj, L.omega_mode); dts = __builtin_fma(B4, dtj, dts); settle(dts); }
            if (PHASE) { ps = __builtin_fma(B4, Y[0] * (any_w ? dtj : 1.0), ps); settle(ps); }
        }
        {
            const double c1 = h * A51, c2 = h * A52, c3 = h * A53, c4 = h * A54;
#pragma unroll
            for (int c = 0; c < 10; ++c)
                Y[c] = __builtin_fma(c4, k4[c], __builtin_fma(c3, k3[c],
                       __builtin_fma(c2, k2[c], __builtin_fma(c1, k1[c], y[c]))));
            rhs<Row, true>(R, u.tc, lb, Y, k5);
            if (__builtin_expect(any_w, 0)) { to_omega_variable(k5, dtj, L.omega_mode); dts = __builtin_fma(B5, dtj, dts); settle(dts); }
            if (PHASE) { ps = __builtin_fma(B5, Y[0] * (any_w ? dtj : 1.0), ps); settle(ps); }
        }
        {
            const double c1 = h * A61, c2 = h * A62, c3 = h * A63, c4 = h * A64, c5 = h * A65;
#pragma unroll
            for (int c = 0; c < 10; ++c)
                Y[c] = __builtin_fma(c5, k5[c], __builtin_fma(c4, k4[c], __builtin_fma(c3, k3[c],
                       __builtin_fma(c2, k2[c], __builtin_fma(c1, k1[c], y[c])))));
            rhs<Row, true>(R, u.tc, lb, Y, k6);
            if (__builtin_expect(any_w, 0)) { to_omega_variable(k6, dtj, L.omega_mode); dts = __builtin_fma(B6, dtj, dts); settle(dts); }
            if (PHASE) { ps = __builtin_fma(B6, Y[0] * (any_w ? dtj : 1.0), ps); settle(ps); }
        }
        // stage 7 point = 5th-order solution; the error sum over k1, k3..k6 is
        // formed now so that those vectors die before the last RHS
        double Ep[10];
        {
            const double c1 = h * B1, c3 = h * B3, c4 = h * B4, c5 = h * B5, c6 = h * B6;
#pragma unroll
            for (int c = 0; c < 10; ++c) {
                Y[c] = __builtin_fma(c6, k6[c], __builtin_fma(c5, k5[c], __builtin_fma(c4, k4[c],
                       __builtin_fma(c3, k3[c], __builtin_fma(c1, k1[c], y[c])))));
                Ep[c] = __builtin_fma(E6, k6[c], __builtin_fma(E5, k5[c], __builtin_fma(E4, k4[c],
                        __builtin_fma(E3, k3[c], E1 * k1[c]))));
            }
        }
        double k7[10], dt7 = 1.0, x7;
        const double lnv7 = rhs_x<Row, true>(R, u.tc, lb, Y, k7, x7);
        if (__builtin_expect(any_w, 0)) to_omega_variable(k7, dt7, L.omega_mode);
        L.nrhs += go ? 6 : 0;

        // the error norm is formed in fixed-step mode too (and ignored there),
        // which keeps it in the same block as its operands
        // the error estimate is h e'; its norm is formed from e' and scaled by h^2
        double e[10];
#pragma unroll
        for (int c = 0; c < 10; ++c) e[c] = __builtin_fma(E7, k7[c], Ep[c]);
        const double z = error_norm(u, y, Y, e) * (h * h);
        bool fin = (GEN && u.fixed) || !__builtin_isnan(z);
#pragma unroll
        for (int c = 0; c < 10; ++c) fin = fin && finite(Y[c]);
        const int acc0 = L.acc;
        const int r = control<RECORD, GEN>(u, L, go, st0, fin, z, h, last, Y, k7, dt7, dts);
        L.lnv = L.acc != acc0 ? lnv7 : L.lnv;
        L.x = L.acc != acc0 ? x7 : L.x;
        if (PHASE) L.phase = L.acc != acc0 ? __builtin_fma(h, ps, L.phase) : L.phase;
        return r;
    }
};

// ===========================================================================
// FP32-split lane
// ===========================================================================
struct LaneF32 {
    double y[10];     // state, FP64
    float k1[10];     // FSAL derivative, FP32
    float dt1;
    double t, h;
    double phase;     // integral of omega dt, FP64 sum of FP32 increments (phase kernels only)
    RowF row;
    int64_t idx;
    int acc, rej, nrhs;
    int nt;           // accepted time steps (unused: no tape in this mode)
    bool omega_mode, last_rej;
    __device__ __forceinline__ double omega() const { return y[0]; }
    __device__ __forceinline__ void set_omega(double w) { y[0] = w; }
    __device__ __forceinline__ void take(const double* Y, const float* k) {
#pragma unroll
        for (int c = 0; c < 10; ++c) {
            y[c] = Y[c];
            k1[c] = k[c];
        }
    }
};

template <bool PHASE = false, bool GEN = true>
struct F32Split {
    using LaneT = LaneF32;

    static __device__ int load(const Io& io, const Uni& u, LaneT& L, int64_t idx) {
        L.idx = idx;
        double m1, m2;
        const int st = read_input<PHASE>(io, u, idx, L.y, m1, m2);
        if (st) return st;
        L.t = 0.0;
        L.acc = 0; L.rej = 0;
        L.omega_mode = false; L.last_rej = false;
        L.h = u.fixed ? u.h_fixed : u.h0;
        L.phase = 0.0;
        Row r;
        make_row(r, m1, m2, u.terms, u.theta_literal);
        L.row = to_f32(r);
        float yf[10];
#pragma unroll
        for (int c = 0; c < 10; ++c) yf[c] = (float)L.y[c];
        rhs_f32(L.row, u.tcf, yf, L.k1);
        L.dt1 = 1.0f;
        L.nrhs = 1;
        return 0;
    }

    static __device__ void finish(const Io& io, const Uni& u, const LaneT& L, int st) {
        write_out<PHASE>(io, u, L.idx, L.y, L.t, L.acc, L.rej, L.nrhs, st, L.phase);
    }

    // One attempted step, run by every lane as in the FP64 lane.
    static __device__ __forceinline__ int step(const Uni& u, LaneT& L, bool active, bool any_w) {
        const int st0 = pre_status<false>(u, L);
        const bool go = active && st0 == 0;
        bool last;
        // idle lanes take a step of zero: their stage points stay on their
        // state, so they never send the wave down a slow path
        const double h = active ? clip_step<GEN>(u, L, last) : 0.0;

        const RowF& R = L.row;
        const float* k1 = L.k1;
        const float hf = (float)h;
        float yf[10], Y[10], k2[10], k3[10], k4[10], k5[10], k6[10];
#pragma unroll
        for (int c = 0; c < 10; ++c) yf[c] = (float)L.y[c];
        float dtj;
        float dts = (float)B1 * L.dt1;
        float ps = 0.0f;
        if (PHASE) ps = (float)B1 * (yf[0] * L.dt1);
        {
            const float c1 = hf * (float)A21;
#pragma unroll
            for (int c = 0; c < 10; ++c) Y[c] = __builtin_fmaf(c1, k1[c], yf[c]);
            rhs_f32(R, u.tcf, Y, k2);
            if (__builtin_expect(any_w, 0)) to_omega_variable(k2, dtj, L.omega_mode);
        }
        {
            const float c1 = hf * (float)A31, c2 = hf * (float)A32;
#pragma unroll
            for (int c = 0; c < 10; ++c) Y[c] = __builtin_fmaf(c2, k2[c], __builtin_fmaf(c1, k1[c], yf[c]));
            rhs_f32(R, u.tcf, Y, k3);
            if (__builtin_expect(any_w, 0)) { to_omega_variable(k3, dtj, L.omega_mode); dts = __builtin_fmaf((float)B3, dtj, dts); settle(dts); }
            if (PHASE) { ps = __builtin_fmaf((float)B3, Y[0] * (any_w ? dtj : 1.0f), ps); settle(ps); }
        }
        {
            const float c1 = hf * (float)A41, c2 = hf * (float)A42, c3 = hf * (float)A43;
#pragma unroll
            for (int c = 0; c < 10; ++c)
                Y[c] = __builtin_fmaf(c3, k3[c], __builtin_fmaf(c2, k2[c], __builtin_fmaf(c1, k1[c], yf[c])));
            rhs_f32(R, u.tcf, Y, k4);
            if (__builtin_expect(any_w, 0)) { to_omega_variable(k4, dtj, L.omega_mode); dts = __builtin_fmaf((float)B4, dtj, dts); settle(dts); }
            if (PHASE) { ps = __builtin_fmaf((float)B4, Y[0] * (any_w ? dtj : 1.0f), ps); settle(ps); }
        }
        {
            const float c1 = hf * (float)A51, c2 = hf * (float)A52, c3 = hf * (float)A53, c4 = hf * (float)A54;
#pragma unroll
            for (int c = 0; c < 10; ++c)
                Y[c] = __builtin_fmaf(c4, k4[c], __builtin_fmaf(c3, k3[c],
                       __builtin_fmaf(c2, k2[c], __builtin_fmaf(c1, k1[c], yf[c]))));
            rhs_f32(R, u.tcf, Y, k5);
            if (__builtin_expect(any_w, 0)) { to_omega_variable(k5, dtj, L.omega_mode); dts = __builtin_fmaf((float)B5, dtj, dts); settle(dts); }
            if (PHASE) { ps = __builtin_fmaf((float)B5, Y[0] * (any_w ? dtj : 1.0f), ps); settle(ps); }
        }
        {
            const float c1 = hf * (float)A61, c2 = hf * (float)A62, c3 = hf * (float)A63, c4 = hf * (float)A64,
                        c5 = hf * (float)A65;
#pragma unroll
            for (int c = 0; c < 10; ++c)
                Y[c] = __builtin_fmaf(c5, k5[c], __builtin_fmaf(c4, k4[c], __builtin_fmaf(c3, k3[c],
                       __builtin_fmaf(c2, k2[c], __builtin_fmaf(c1, k1[c], yf[c])))));
            rhs_f32(R, u.tcf, Y, k6);
            if (__builtin_expect(any_w, 0)) { to_omega_variable(k6, dtj, L.omega_mode); dts = __builtin_fmaf((float)B6, dtj, dts); settle(dts); }
            if (PHASE) { ps = __builtin_fmaf((float)B6, Y[0] * (any_w ? dtj : 1.0f), ps); settle(ps); }
        }
        // 5th-order increment D (FP32), the stage-7 point, and the error sum
        float D[10], Ep[10];
#pragma unroll
        for (int c = 0; c < 10; ++c) {
            D[c] = hf * __builtin_fmaf((float)B6, k6[c], __builtin_fmaf((float)B5, k5[c],
                        __builtin_fmaf((float)B4, k4[c], __builtin_fmaf((float)B3, k3[c], (float)B1 * k1[c]))));
            Y[c] = yf[c] + D[c];
            Ep[c] = __builtin_fmaf((float)E6, k6[c], __builtin_fmaf((float)E5, k5[c],
                    __builtin_fmaf((float)E4, k4[c], __builtin_fmaf((float)E3, k3[c], (float)E1 * k1[c]))));
        }
        float k7[10], dt7 = 1.0f;
        rhs_f32(R, u.tcf, Y, k7);
        if (__builtin_expect(any_w, 0)) to_omega_variable(k7, dt7, L.omega_mode);
        L.nrhs += go ? 6 : 0;

        // candidate state in FP64
        double ynew[10];
#pragma unroll
        for (int c = 0; c < 10; ++c) ynew[c] = L.y[c] + (double)D[c];
        double e[10];
#pragma unroll
        for (int c = 0; c < 10; ++c) e[c] = (double)(hf * __builtin_fmaf((float)E7, k7[c], Ep[c]));
        const double z = error_norm_pairs(u, L.y, ynew, e);
        bool fin = (GEN && u.fixed) || !__builtin_isnan(z);
#pragma unroll
        for (int c = 0; c < 10; ++c) fin = fin && finite(ynew[c]) && __builtin_isfinite(k7[c]);
        const int acc0 = L.acc;
        const int r = control<false, GEN>(u, L, go, st0, fin, z, h, last, ynew, k7, dt7, dts);
        // the FP32 increment is summed in FP64, as the state is
        if (PHASE) L.phase = L.acc != acc0 ? __builtin_fma(h, (double)ps, L.phase) : L.phase;
        return r;
    }
};

// ===========================================================================
// FP32-state lane
// ===========================================================================
// Sum a + b of two floats as hi + lo exactly (Fast2Sum: requires |a| >= |b|
// or a = 0; here a is the running sum and b one step's increment).
__device__ __forceinline__ void fast_two_sum(float a, float b, float& hi, float& lo) {
    hi = a + b;
    lo = b - (hi - a);
}

struct LaneF32S {
    float y[10];      // state, FP32; omega is y[0] + wlo
    float wlo;        // low part of omega: the rounding of its increments, summed
    float k1[10];     // FSAL derivative, FP32
    float dt1;
    double t, h;
    float ph, phlo;   // orbital phase as ph + phlo (phase kernels only)
    RowF row;
    int64_t idx;
    int acc, rej, nrhs;
    int nt;           // accepted time steps (unused: no tape in this mode)
    bool omega_mode, last_rej;
    __device__ __forceinline__ double omega() const { return (double)y[0] + (double)wlo; }
    // omega as the nearest float and the float nearest the rest (exact for
    // the values this lane produces: a float plus a float below half its ulp)
    __device__ __forceinline__ void set_omega(double w) {
        y[0] = (float)w;
        wlo = (float)(w - (double)y[0]);
    }
    __device__ __forceinline__ void take(const double* Y, const float* k) {
        set_omega(Y[0]);
#pragma unroll
        for (int c = 1; c < 10; ++c) y[c] = (float)Y[c];
#pragma unroll
        for (int c = 0; c < 10; ++c) k1[c] = k[c];
    }
    __device__ __forceinline__ void state64(double* yd) const {
        yd[0] = omega();
#pragma unroll
        for (int c = 1; c < 10; ++c) yd[c] = (double)y[c];
    }
};

// FP32 state (Sec. III: single precision with a few computations in double):
// omega, S1, S2 and L_hat are held in FP32, with the increments of omega
// summed with their rounding errors (omega = y[0] + wlo, about 48 bits) and
// likewise the phase; the stages, right-hand sides, increments and error
// estimate are FP32; t, h, the error norm, the step control and the
// omega >= omega_f test are FP64.
template <bool PHASE = false, bool GEN = true>
struct F32State {
    using LaneT = LaneF32S;

    static __device__ int load(const Io& io, const Uni& u, LaneT& L, int64_t idx) {
        L.idx = idx;
        double m1, m2, yd[10];
        const int st = read_input<PHASE>(io, u, idx, yd, m1, m2);
        if (st) return st;
        L.set_omega(yd[0]);
#pragma unroll
        for (int c = 1; c < 10; ++c) L.y[c] = (float)yd[c];
        L.t = 0.0;
        L.acc = 0; L.rej = 0;
        L.omega_mode = false; L.last_rej = false;
        L.h = u.fixed ? u.h_fixed : u.h0;
        L.ph = 0.0f;
        L.phlo = 0.0f;
        Row r;
        make_row(r, m1, m2, u.terms, u.theta_literal);
        L.row = to_f32(r);
        rhs_f32(L.row, u.tcf, L.y, L.k1);
        L.dt1 = 1.0f;
        L.nrhs = 1;
        return 0;
    }

    static __device__ void finish(const Io& io, const Uni& u, const LaneT& L, int st) {
        double yd[10];
        L.state64(yd);
        // an integration that reached omega_f ends on it exactly (the float
        // pair holds 48 bits of it)
        if (st == PN_ST_OK && !u.tend) yd[0] = u.omega_f;
        write_out<PHASE>(io, u, L.idx, yd, L.t, L.acc, L.rej, L.nrhs, st, (double)L.ph + (double)L.phlo);
    }

    // One attempted step, run by every lane as in the FP64 lane.
    static __device__ __forceinline__ int step(const Uni& u, LaneT& L, bool active, bool any_w) {
        const int st0 = pre_status<false>(u, L);
        const bool go = active && st0 == 0;
        bool last;
        // idle lanes take a step of zero: their stage points stay on their
        // state, so they never send the wave down a slow path
        const double h = active ? clip_step<GEN>(u, L, last) : 0.0;

        const RowF& R = L.row;
        const float* k1 = L.k1;
        const float* yf = L.y;
        const float hf = (float)h;
        float Y[10], k2[10], k3[10], k4[10], k5[10], k6[10];
        float dtj;
        float dts = (float)B1 * L.dt1;
        float ps = 0.0f;
        if (PHASE) ps = (float)B1 * (yf[0] * L.dt1);
        {
            const float c1 = hf * (float)A21;
#pragma unroll
            for (int c = 0; c < 10; ++c) Y[c] = __builtin_fmaf(c1, k1[c], yf[c]);
            rhs_f32(R, u.tcf, Y, k2);
            if (__builtin_expect(any_w, 0)) to_omega_variable(k2, dtj, L.omega_mode);
        }
        {
            const float c1 = hf * (float)A31, c2 = hf * (float)A32;
#pragma unroll
            for (int c = 0; c < 10; ++c) Y[c] = __builtin_fmaf(c2, k2[c], __builtin_fmaf(c1, k1[c], yf[c]));
            rhs_f32(R, u.tcf, Y, k3);
            if (__builtin_expect(any_w, 0)) { to_omega_variable(k3, dtj, L.omega_mode); dts = __builtin_fmaf((float)B3, dtj, dts); settle(dts); }
            if (PHASE) { ps = __builtin_fmaf((float)B3, Y[0] * (any_w ? dtj : 1.0f), ps); settle(ps); }
        }
        {
            const float c1 = hf * (float)A41, c2 = hf * (float)A42, c3 = hf * (float)A43;
#pragma unroll
            for (int c = 0; c < 10; ++c)
                Y[c] = __builtin_fmaf(c3, k3[c], __builtin_fmaf(c2, k2[c], __builtin_fmaf(c1, k1[c], yf[c])));
            rhs_f32(R, u.tcf, Y, k4);
            if (__builtin_expect(any_w, 0)) { to_omega_variable(k4, dtj, L.omega_mode); dts = __builtin_fmaf((float)B4, dtj, dts); settle(dts); }
            if (PHASE) { ps = __builtin_fmaf((float)B4, Y[0] * (any_w ? dtj : 1.0f), ps); settle(ps); }
        }
        {
            const float c1 = hf * (float)A51, c2 = hf * (float)A52, c3 = hf * (float)A53, c4 = hf * (float)A54;
#pragma unroll
            for (int c = 0; c < 10; ++c)
                Y[c] = __builtin_fmaf(c4, k4[c], __builtin_fmaf(c3, k3[c],
                       __builtin_fmaf(c2, k2[c], __builtin_fmaf(c1, k1[c], yf[c]))));
            rhs_f32(R, u.tcf, Y, k5);
            if (__builtin_expect(any_w, 0)) { to_omega_variable(k5, dtj, L.omega_mode); dts = __builtin_fmaf((float)B5, dtj, dts); settle(dts); }
            if (PHASE) { ps = __builtin_fmaf((float)B5, Y[0] * (any_w ? dtj : 1.0f), ps); settle(ps); }
        }
        {
            const float c1 = hf * (float)A61, c2 = hf * (float)A62, c3 = hf * (float)A63, c4 = hf * (float)A64,
                        c5 = hf * (float)A65;
#pragma unroll
            for (int c = 0; c < 10; ++c)
                Y[c] = __builtin_fmaf(c5, k5[c], __builtin_fmaf(c4, k4[c], __builtin_fmaf(c3, k3[c],
                       __builtin_fmaf(c2, k2[c], __builtin_fmaf(c1, k1[c], yf[c])))));
            rhs_f32(R, u.tcf, Y, k6);
            if (__builtin_expect(any_w, 0)) { to_omega_variable(k6, dtj, L.omega_mode); dts = __builtin_fmaf((float)B6, dtj, dts); settle(dts); }
            if (PHASE) { ps = __builtin_fmaf((float)B6, Y[0] * (any_w ? dtj : 1.0f), ps); settle(ps); }
        }
        // 5th-order increment D (FP32), the stage-7 point, and the error sum
        float D[10], Ep[10];
#pragma unroll
        for (int c = 0; c < 10; ++c) {
            D[c] = hf * __builtin_fmaf((float)B6, k6[c], __builtin_fmaf((float)B5, k5[c],
                        __builtin_fmaf((float)B4, k4[c], __builtin_fmaf((float)B3, k3[c], (float)B1 * k1[c]))));
            Y[c] = yf[c] + D[c];
            Ep[c] = __builtin_fmaf((float)E6, k6[c], __builtin_fmaf((float)E5, k5[c],
                    __builtin_fmaf((float)E4, k4[c], __builtin_fmaf((float)E3, k3[c], (float)E1 * k1[c]))));
        }
        float k7[10], dt7 = 1.0f;
        rhs_f32(R, u.tcf, Y, k7);
        if (__builtin_expect(any_w, 0)) to_omega_variable(k7, dt7, L.omega_mode);
        L.nrhs += go ? 6 : 0;

        // the state and the candidate, viewed in FP64 for the norm and the
        // control: omega's increment joins the compensated sum, the other
        // components are the FP32 sums already formed
        double yd[10], ynew[10];
        L.state64(yd);
        float whi, wlo;
        fast_two_sum(yf[0], D[0], whi, wlo);
        ynew[0] = (double)whi + (double)(wlo + L.wlo);
#pragma unroll
        for (int c = 1; c < 10; ++c) ynew[c] = (double)Y[c];
        double e[10];
#pragma unroll
        for (int c = 0; c < 10; ++c) e[c] = (double)(hf * __builtin_fmaf((float)E7, k7[c], Ep[c]));
        const double z = error_norm_each(u, yd, ynew, e);
        bool fin = (GEN && u.fixed) || !__builtin_isnan(z);
#pragma unroll
        for (int c = 0; c < 10; ++c) fin = fin && finite(ynew[c]) && __builtin_isfinite(k7[c]);
        const int acc0 = L.acc;
        const int r = control<false, GEN>(u, L, go, st0, fin, z, h, last, ynew, k7, dt7, dts);
        if (PHASE && L.acc != acc0) {
            // the phase increment joins its compensated sum
            float s, err;
            fast_two_sum(L.ph, hf * ps, s, err);
            L.ph = s;
            L.phlo += err;
        }
        return r;
    }
};

// ===========================================================================
// Scheduling
// ===========================================================================
__device__ __forceinline__ int lane_id() { return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u)); }

__device__ __forceinline__ uint64_t wave_ballot(bool p) { return __ballot(p); }

// Persistent loop: each wave hands new inspirals to idle lanes from a global
// counter, until the counter passes n and its lanes are done.  A lane that
// finishes keeps its final state and status until the wave's next refill
// pass, which first writes the outputs of all such lanes at once (the output
// code then runs once per pass rather than once per finishing step); once
// the counter is exhausted, every iteration with an idle lane is such a
// pass, so the last outputs are written before the wave exits.
template <class P>
__device__ __forceinline__ void persistent_loop(const Uni& u, unsigned long long* slot) {
    const int lane = lane_id();
    unsigned long long* counter = slot;
    typename P::LaneT L{};      // idle lanes step on this state and discard the result
    L.y[0] = 1.0;               // a positive omega keeps their arithmetic finite
    bool active = false;
    // A finished lane whose outputs are not yet written keeps its status in
    // L.h, which it no longer needs: L.h = -(status + kPend) < 0 (statuses
    // are 1 and -1 .. -6; a lane that is idle otherwise has L.h >= 0).
    constexpr int kPend = 16;
    bool exhausted = false;     // wave-uniform
    for (;;) {
        uint64_t need = wave_ballot(!active);
        const int nidle = __popcll(need);
        if (need != 0 && (exhausted || nidle >= u.refill_min || nidle == 64)) {
            // The inputs, outputs and the arguments only a refill needs are read
            // from the launch descriptor in the call's slot here, rather than
            // kept in scalar registers across the step loop, which needs them all.
            const LaunchDesc* d = reinterpret_cast<const LaunchDesc*>(slot + kDescOffset);
            asm volatile("" : "+s"(d));        // keep the loads inside the pass
            const Io& io = d->io;
            const Uni& uc = d->u;
            // ---- outputs of the lanes that finished since the last pass ------------
            if (!active && L.h < 0.0) {
                const int r = -(int)L.h - kPend;
                P::finish(io, uc, L, r == 1 ? PN_ST_OK : r);
                L.h = 0.0;
            }
            // ---- refill idle lanes ------------------------------------------------
            while (need != 0 && !exhausted) {
                const int cnt = __popcll(need);
                const int leader = __ffsll((unsigned long long)need) - 1;
                unsigned long long base = 0;
                if (lane == leader) base = atomicAdd(counter, (unsigned long long)cnt);
                const unsigned lo = __builtin_amdgcn_readlane((unsigned)(base & 0xffffffffu), leader);
                const unsigned hi = __builtin_amdgcn_readlane((unsigned)(base >> 32), leader);
                base = ((unsigned long long)hi << 32) | lo;
                bool still = false;
                if (!active) {
                    const unsigned rank = __builtin_amdgcn_mbcnt_hi((unsigned)(need >> 32),
                                          __builtin_amdgcn_mbcnt_lo((unsigned)need, 0u));
                    const unsigned long long pos = base + rank;
                    if (pos < (unsigned long long)u.n) {
                        const int64_t idx = io.order ? (int64_t)io.order[pos] : (int64_t)pos;
                        if (idx >= 0 && idx < u.n) {
                            const int st = P::load(io, uc, L, idx);
                            if (st == 0) active = true; else still = true;
                        } else {
                            still = true;      // not an index: this slot integrates nothing
                        }
                    }
                }
                if (base + cnt >= (unsigned long long)u.n) exhausted = true;
                need = wave_ballot(still);
            }
        }
        if (wave_ballot(active) == 0) {
            if (exhausted) break;
            continue;
        }
        // ---- one step on every active lane ----------------------------------------
        // A lane in omega-mode takes its last step (usually one) only once the
        // wave has enough such lanes and idle lanes to refill right after; it
        // waits until then as an idle lane would, so that the omega-mode
        // arithmetic runs in fewer wave-steps.
        const uint64_t wmask = wave_ballot(active && L.omega_mode);
        const uint64_t amask = wave_ballot(active);
        const bool run_w = wmask != 0 && (exhausted || wmask == amask ||
                                          __popcll(wmask) + (64 - __popcll(amask)) >= u.refill_min);
        const bool act = active && (run_w || !L.omega_mode);
        const int r = P::step(u, L, act, run_w);
        if (act && r != 0) {
            L.h = -(double)(r + kPend);
            active = false;
        }
    }
}

// One lane per inspiral, no refill: a wave runs until its longest inspiral ends.
template <class P>
__device__ __forceinline__ void static_loop(const Io& io, const Uni& u, int64_t pos) {
    typename P::LaneT L{};
    L.y[0] = 1.0;
    bool active = false;
    if (pos < u.n) {
        const int64_t idx = io.order ? (int64_t)io.order[pos] : pos;
        if (idx >= 0 && idx < u.n) active = P::load(io, u, L, idx) == 0;
    }
    for (;;) {
        if (wave_ballot(active) == 0) break;
        const bool any_w = wave_ballot(active && L.omega_mode) != 0;
        const int r = P::step(u, L, active, any_w);
        if (active && r != 0) {
            P::finish(io, u, L, r == 1 ? PN_ST_OK : r);
            active = false;
        }
    }
}

template <int BLOCK, bool RECORD>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(kWpeF64)))
void integrate_persistent_f64(Uni u, unsigned long long* slot) {
    persistent_loop<F64<RECORD, false, false>>(u, slot);      // adaptive, to omega_f
}

template <int BLOCK, bool RECORD>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(kWpeF64)))
void integrate_persistent_f64_modes(Uni u, unsigned long long* slot) {
    persistent_loop<F64<RECORD, false, true>>(u, slot);       // also fixed step and t_end
}

template <int BLOCK>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(kWpeF32)))
void integrate_persistent_f32s(Uni u, unsigned long long* slot) {
    persistent_loop<F32Split<false, false>>(u, slot);
}

template <int BLOCK>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(kWpeF32)))
void integrate_persistent_f32s_modes(Uni u, unsigned long long* slot) {
    persistent_loop<F32Split<false, true>>(u, slot);
}

// the same loops with the orbital phase integrated alongside
template <int BLOCK>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(kWpeF64)))
void integrate_persistent_f64_phase(Uni u, unsigned long long* slot) {
    persistent_loop<F64<false, true>>(u, slot);
}

template <int BLOCK>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(kWpeF32)))
void integrate_persistent_f32s_phase(Uni u, unsigned long long* slot) {
    persistent_loop<F32Split<true>>(u, slot);
}

template <int BLOCK>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(kWpeF32S)))
void integrate_persistent_f32x(Uni u, unsigned long long* slot) {
    persistent_loop<F32State<false, false>>(u, slot);
}

template <int BLOCK>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(kWpeF32S)))
void integrate_persistent_f32x_modes(Uni u, unsigned long long* slot) {
    persistent_loop<F32State<false, true>>(u, slot);
}

template <int BLOCK>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(kWpeF32S)))
void integrate_persistent_f32x_phase(Uni u, unsigned long long* slot) {
    persistent_loop<F32State<true>>(u, slot);
}

template <int BLOCK>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(kWpeF32S)))
void integrate_static_f32x(Io io, Uni u) {
    static_loop<F32State<>>(io, u, (int64_t)blockIdx.x * BLOCK + threadIdx.x);
}

template <int BLOCK>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(kWpeF32S)))
void integrate_static_f32x_phase(Io io, Uni u) {
    static_loop<F32State<true>>(io, u, (int64_t)blockIdx.x * BLOCK + threadIdx.x);
}

template <int BLOCK, bool RECORD>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(kWpeF64)))
void integrate_static_f64(Io io, Uni u) {
    static_loop<F64<RECORD>>(io, u, (int64_t)blockIdx.x * BLOCK + threadIdx.x);
}

template <int BLOCK>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(kWpeF32)))
void integrate_static_f32s(Io io, Uni u) {
    static_loop<F32Split<>>(io, u, (int64_t)blockIdx.x * BLOCK + threadIdx.x);
}

template <int BLOCK>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(kWpeF64)))
void integrate_static_f64_phase(Io io, Uni u) {
    static_loop<F64<false, true>>(io, u, (int64_t)blockIdx.x * BLOCK + threadIdx.x);
}

template <int BLOCK>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(kWpeF32)))
void integrate_static_f32s_phase(Io io, Uni u) {
    static_loop<F32Split<true>>(io, u, (int64_t)blockIdx.x * BLOCK + threadIdx.x);
}

// ===========================================================================
// Discrete adjoint (reverse mode of the replayed FP64 Dormand-Prince map)
// ===========================================================================
//
// The forward map, with the recorded step sizes frozen: n_t time steps
// y <- Phi_f(y, h_k), then n_w steps in omega, z = (t, y) <- Phi_g(z, D_j),
// g = (1/f_0, 1, f_1/f_0, ..., f_9/f_0), the last D = omega_f - omega.  The
// backward pass walks the checkpoint segments from the last one: it replays
// K steps forward from the checkpoint (states into the workspace), then
// runs the RK adjoint recurrence through them in reverse:
//   Lambda_i = h (b_i lambda_{n+1} + sum_{j>i} a_ji mu_j),  mu_i = J(Y_i)^T Lambda_i,
//   lambda_n = lambda_{n+1} + sum_i mu_i,
// plus dL/dD * dD/domega_n = -dL/dD for the last omega-step.

struct AdjUni {
    double omega_f;
    TermConsts tc;
    int64_t n, ld;
    int terms, theta_literal;
    const double* tape;
    int64_t tape_stride;
    int tape_cap, ckpt_every;
};

struct AdjIo {
    const double* __restrict__ m;
    const int32_t* __restrict__ status;
    const double* __restrict__ gy;      // [10][ld]
    const double* __restrict__ gt;      // [ld] or null
    double* __restrict__ g_m;           // [2][ld]
    double* __restrict__ g_S0;          // [6][ld]
    double* __restrict__ g_L0;          // [3][ld]
    double* __restrict__ g_w0;          // [ld]
    double* __restrict__ ws;            // [K][11][n]: per grid lane, the segment's states and steps
    const int32_t* __restrict__ order;  // [n] or null
};

// the stage derivative: f (time mode) or g (omega mode); the cube root and
// log of the stage from the step's base point lb
__device__ __forceinline__ void stage_deriv(const Row& R, const TermConsts& tc, const LogBase& lb, const double* Y,
                                            double* k, bool om) {
    rhs<Row, true>(R, tc, lb, Y, k);
    if (om) {
        const double s = 1.0 / k[0];
#pragma unroll
        for (int c = 1; c < 10; ++c) k[c] *= s;
        k[0] = 1.0;
    }
}

// one replayed step (no error control): y <- y + h sum b_i k_i
__device__ __forceinline__ void replay_step(const Row& R, const TermConsts& tc, double* y, double h, bool om) {
    double k1[10], k2[10], k3[10], k4[10], k5[10], k6[10], Y[10];
    const LogBase lb = log_base(R, y);
    stage_deriv(R, tc, lb, y, k1, om);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int c = 0; c < 10; ++c) Y[c] = __builtin_fma(h * A21, k1[c], y[c]);
    stage_deriv(R, tc, lb, Y, k2, om);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int c = 0; c < 10; ++c) Y[c] = __builtin_fma(h * A32, k2[c], __builtin_fma(h * A31, k1[c], y[c]));
    stage_deriv(R, tc, lb, Y, k3, om);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int c = 0; c < 10; ++c)
        Y[c] = __builtin_fma(h * A43, k3[c], __builtin_fma(h * A42, k2[c], __builtin_fma(h * A41, k1[c], y[c])));
    stage_deriv(R, tc, lb, Y, k4, om);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int c = 0; c < 10; ++c)
        Y[c] = __builtin_fma(h * A54, k4[c], __builtin_fma(h * A53, k3[c],
               __builtin_fma(h * A52, k2[c], __builtin_fma(h * A51, k1[c], y[c]))));
    stage_deriv(R, tc, lb, Y, k5, om);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int c = 0; c < 10; ++c)
        Y[c] = __builtin_fma(h * A65, k5[c], __builtin_fma(h * A64, k4[c], __builtin_fma(h * A63, k3[c],
               __builtin_fma(h * A62, k2[c], __builtin_fma(h * A61, k1[c], y[c])))));
    stage_deriv(R, tc, lb, Y, k6, om);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int c = 0; c < 10; ++c)
        y[c] = __builtin_fma(h * B6, k6[c], __builtin_fma(h * B5, k5[c], __builtin_fma(h * B4, k4[c],
               __builtin_fma(h * B3, k3[c], __builtin_fma(h * B1, k1[c], y[c])))));
}

// Reverse of one step.  lam (10) and the row adjoint are updated in place;
// lt is dL/dt (constant along the path).  `last` marks the last omega-step,
// whose size D = omega_f - omega depends on the state: it adds -dL/dD to
// lam[0].
//   ys: this lane's LDS rows, entry (s, c) at ys[(s * 10 + c) * 64]: the state
//       before the step (slot 0, filled by the caller), the stage points
//       Y_2..Y_6 (slots 1..5; each replaced by its stage adjoint mu_j once
//       stage j is reversed), and the step's log base (slot 6, entries 0..3);
//   pf: the state and step size of the step reversed next (workspace column,
//       entry c at pf[c * pfstride]), parked in nx (LDS, entry c at nx[c * 64]).
// What stays in registers across the stages is the row, its adjoint, lambda
// and the stage being reversed: at one wave per SIMD these fit in the 256
// VGPRs and the AGPRs without scratch.
__device__ __forceinline__ void reverse_step(const Row& R, const TermConsts& tc, double h, bool om, bool last,
                                             double* lam, double lt, RowBar& rb, double* __restrict__ ys,
                                             const double* __restrict__ pf, int64_t pfstride,
                                             double* __restrict__ nx) {
#define YS(S, C) ys[((S) * 10 + (C)) * 64]
    // mu_j (j = 2..6) goes to the LDS slot of Y_j once stage j is reversed
    // (Y_j is dead then) and is read back through a pointer the compiler
    // cannot see through (the empty asm after each stage), so that the
    // values are not kept in registers instead
    typedef __attribute__((address_space(3))) double lds_double;
    lds_double* ml = (lds_double*)ys;
#define MS(J, C) ml[(((J) + 1) * 10 + (C)) * 64]
    const LogBase lb{};
    {
        double y[10];
#pragma unroll
        for (int c = 0; c < 10; ++c) y[c] = YS(0, c);
        // the next reverse step's state and step size: loaded now, stored to
        // LDS once the stage points are formed, so that the load latency
        // overlaps the recomputation instead of opening the next step
        double nxt[11];
#pragma unroll
        for (int c = 0; c < 11; ++c) nxt[c] = pf[c * pfstride];
        double k1[10], k2[10], k3[10], k4[10], k5[10], Y[10];
        const LogBase lbs = log_base(R, y);
        YS(6, 0) = lbs.lnv; YS(6, 1) = lbs.x; YS(6, 2) = lbs.w; YS(6, 3) = lbs.iw;
        stage_deriv(R, tc, lbs, y, k1, om);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int c = 0; c < 10; ++c) { Y[c] = __builtin_fma(h * A21, k1[c], y[c]); YS(1, c) = Y[c]; }
        stage_deriv(R, tc, lbs, Y, k2, om);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int c = 0; c < 10; ++c) {
            Y[c] = __builtin_fma(h * A32, k2[c], __builtin_fma(h * A31, k1[c], y[c]));
            YS(2, c) = Y[c];
        }
        stage_deriv(R, tc, lbs, Y, k3, om);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int c = 0; c < 10; ++c) {
            Y[c] = __builtin_fma(h * A43, k3[c], __builtin_fma(h * A42, k2[c], __builtin_fma(h * A41, k1[c], y[c])));
            YS(3, c) = Y[c];
        }
        stage_deriv(R, tc, lbs, Y, k4, om);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int c = 0; c < 10; ++c) {
            Y[c] = __builtin_fma(h * A54, k4[c], __builtin_fma(h * A53, k3[c],
                   __builtin_fma(h * A52, k2[c], __builtin_fma(h * A51, k1[c], y[c]))));
            YS(4, c) = Y[c];
        }
        stage_deriv(R, tc, lbs, Y, k5, om);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int c = 0; c < 10; ++c)
            YS(5, c) = __builtin_fma(h * A65, k5[c], __builtin_fma(h * A64, k4[c],
                       __builtin_fma(h * A63, k3[c], __builtin_fma(h * A62, k2[c],
                       __builtin_fma(h * A61, k1[c], y[c])))));
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int c = 0; c < 11; ++c) nx[c * 64] = nxt[c];
    }

    // reverse: stage i = 6 .. 1; mu_j (j > i) read back from LDS
    double mu1[10];      // mu_1 (the others are in LDS)
    double dh = 0.0;     // dL/dh (last omega-step only)

    // Lh = b_i lam + sum_{j>i} a_ji mu_j ; the VJP is seeded with h Lh
#define PN_REV_STAGE(SLOT, BI, MUJ, LAMEXPR)                                                      \
    {                                                                                            \
        double Yi[10], Lh[10], mu[10];                                                           \
        _Pragma("unroll") for (int c = 0; c < 10; ++c) {                                         \
            Yi[c] = YS(SLOT, c);                                                                 \
            Lh[c] = (LAMEXPR);                                                                   \
        }                                                                                        \
        const LogBase lbv{ml[(60) * 64], ml[(61) * 64], ml[(62) * 64], ml[(63) * 64]};              \
        rhs_vjp(R, tc, lbv, Yi, Lh, h, lt * h * (BI), om, mu, rb);                                       \
        /* the row adjoint's updates are completed here: left to itself the */                 \
        /* compiler defers them to the end of the step and keeps every */                         \
        /* stage's operands alive until then (~700 AGPR moves and scratch */                      \
        /* spills per step) */                                                                   \
        _Pragma("unroll") for (int i = 0; i < NROW; ++i) settle(rb.v[i]);                          \
        if (last) {                                                                              \
            double f[10];                                                                        \
            rhs<Row, false>(R, tc, lb, Yi, f);                                                   \
            const double s = 1.0 / f[0];                                                         \
            double dot = Lh[0];                                                                  \
            _Pragma("unroll") for (int c = 1; c < 10; ++c) dot = __builtin_fma(f[c] * s, Lh[c], dot); \
            dh += dot + lt * (BI) * s;                                                           \
        }                                                                                        \
        _Pragma("unroll") for (int c = 0; c < 10; ++c) {                                         \
            if ((MUJ) < 0) mu1[c] = mu[c];                                                       \
            if ((MUJ) >= 0) MS((MUJ) >= 0 ? (MUJ) : 0, c) = mu[c];                               \
        }                                                                                        \
        __asm__ volatile("" : "+v"(ml));                                                          \
        __builtin_amdgcn_sched_barrier(0);                                                       \
    }

    PN_REV_STAGE(5, B6, 4, B6 * lam[c])
    PN_REV_STAGE(4, B5, 3, __builtin_fma(A65, MS(4, c), B5 * lam[c]))
    PN_REV_STAGE(3, B4, 2, __builtin_fma(A64, MS(4, c), __builtin_fma(A54, MS(3, c), B4 * lam[c])))
    PN_REV_STAGE(2, B3, 1, __builtin_fma(A63, MS(4, c), __builtin_fma(A53, MS(3, c),
                             __builtin_fma(A43, MS(2, c), B3 * lam[c]))))
    PN_REV_STAGE(1, 0.0, 0, __builtin_fma(A62, MS(4, c), __builtin_fma(A52, MS(3, c),
                              __builtin_fma(A42, MS(2, c), A32 * MS(1, c)))))
    PN_REV_STAGE(0, B1, -1, __builtin_fma(A61, MS(4, c), __builtin_fma(A51, MS(3, c), __builtin_fma(A41, MS(2, c),
                              __builtin_fma(A31, MS(1, c), __builtin_fma(A21, MS(0, c), B1 * lam[c]))))))
#undef PN_REV_STAGE
    // lambda_n = lambda_{n+1} + mu_6 + ... + mu_1 (in the order the stages are reversed)
#pragma unroll
    for (int c = 0; c < 10; ++c)
        lam[c] = ((((lam[c] + MS(4, c)) + MS(3, c)) + MS(2, c)) + MS(1, c)) + MS(0, c) + mu1[c];
#undef YS
#undef MS

    if (last) lam[0] -= dh;
}

// wsl: this grid lane's column of the segment workspace, entry (k, c) at
// wsl[(k * 11 + c) * n] (c < 10: the state before step k of the segment,
// c = 10: that step's size), so that a wave's accesses are coalesced.
__device__ void adjoint_one(const AdjIo& io, const AdjUni& u, int64_t idx, double* wsl, double* ys, double* nx) {
    const int64_t ld = u.ld;
    const int st = io.status[idx];
    const double* tp = u.tape + idx * u.tape_stride;
    double lam[10];
#pragma unroll
    for (int c = 0; c < 10; ++c) lam[c] = io.gy[c * ld + idx];
    // the step counts of the tape must be those of a recorded run: integers
    // with n_t + n_w <= cap (else the tape is not read beyond its row)
    const double tnt = tp[0], tnw = tp[1];
    const bool tape_ok = tnt >= 0.0 && tnw >= 0.0 && tnt + tnw <= (double)u.tape_cap &&
                         tnt == __builtin_floor(tnt) && tnw == __builtin_floor(tnw);
    if (st == PN_ST_DONE_AT_START || st != PN_ST_OK || !tape_ok) {
        // done at start: the output is the input; failures: no gradient
        const double fill = (st == PN_ST_DONE_AT_START) ? 1.0 : __builtin_nan("");   // (a bad tape: NaN)
        io.g_m[idx] = st == PN_ST_DONE_AT_START ? 0.0 : fill;
        io.g_m[ld + idx] = st == PN_ST_DONE_AT_START ? 0.0 : fill;
        io.g_w0[idx] = lam[0] * fill;
#pragma unroll
        for (int c = 0; c < 6; ++c) io.g_S0[c * ld + idx] = lam[1 + c] * fill;
#pragma unroll
        for (int c = 0; c < 3; ++c) io.g_L0[c * ld + idx] = lam[7 + c] * fill;
        return;
    }
    const double m1 = io.m[idx], m2 = io.m[ld + idx];
    Row R;
    make_row(R, m1, m2, u.terms, u.theta_literal);
    RowBar rb;
#pragma unroll
    for (int i = 0; i < NROW; ++i) rb.v[i] = 0.0;
    const double lt = io.gt ? io.gt[idx] : 0.0;
    const int nt = (int)tnt;
    const int N = nt + (int)tnw;
    const int K = u.ckpt_every;
    const double* hs = tp + 2;
    const double* ck = tp + 2 + u.tape_cap;
    const int64_t wstride = u.n;
#define WS(K_, C_) wsl[((int64_t)(K_) * 11 + (C_)) * wstride]
    const int nseg = (N + K - 1) / K;
    // The lanes of a wave walk their segments in step: iteration sg handles
    // segment sg on every lane that has one, counting down from the wave's
    // largest segment count.  Counting down from each lane's own count would
    // pair one lane's short last segment with another's full one, and a wave
    // whose lanes straddle a multiple of K would take up to ~1.5x its longest
    // inspiral.  The wave maximum is taken bit by bit with ballots, over the
    // lanes still running (those that returned above take no part).
    int nmax = 0;
    for (int b = 28; b >= 0; --b) {        // nseg <= cap_steps <= 2^28
        const int cand = nmax | (1 << b);
        if (__ballot(nseg >= cand) != 0) nmax = cand;
    }
    for (int sg = nmax - 1; sg >= 0; --sg) {
        if (sg >= nseg) continue;           // this lane has no segment sg
        const int k0 = sg * K;
        const int k1 = (k0 + K < N) ? k0 + K : N;
        double y[10];
#pragma unroll
        for (int c = 0; c < 10; ++c) y[c] = ck[(int64_t)sg * 10 + c];
        double hk = hs[k0];
        for (int k = k0; k < k1; ++k) {
            const bool om = k >= nt;
            const double h = (om && k == N - 1) ? u.omega_f - y[0] : hk;
            if (k + 1 < k1) {
                hk = hs[k + 1];                   // loaded a step ahead
#pragma unroll
                for (int c = 0; c < 10; ++c) WS(k - k0, c) = y[c];
                WS(k - k0, 10) = h;
                replay_step(R, u.tc, y, h, om);   // the state after the segment is not needed
            } else {
                // the segment's last step is reversed first: straight to LDS
#pragma unroll
                for (int c = 0; c < 10; ++c) nx[c * 64] = y[c];
                nx[10 * 64] = h;
            }
        }
        for (int k = k1 - 1; k >= k0; --k) {
#pragma unroll
            for (int c = 0; c < 10; ++c) ys[c * 64] = nx[c * 64];
            const double h = nx[10 * 64];
            const bool om = k >= nt;
            const bool last = om && k == N - 1;
            // the step reversed next (k - 1; at k0 a valid row, not used)
            const double* pf = &WS((k > k0 ? k - 1 : k0) - k0, 0);
            reverse_step(R, u.tc, h, om, last, lam, lt, rb, ys, pf, wstride, nx);
        }
    }
#undef WS
    // chain the row adjoint to the masses
    double gm[2];
#pragma unroll
    for (int dir = 0; dir < 2; ++dir) {
        RowDual rd;
        make_row_dual(rd, Dl(m1, dir == 0 ? 1.0 : 0.0), Dl(m2, dir == 1 ? 1.0 : 0.0), u.terms, u.theta_literal);
        double g = 0.0;
#pragma unroll
        for (int i = 0; i < NROW; ++i) g = __builtin_fma(rb.v[i], rd.v[i].d, g);
        gm[dir] = g;
    }
    io.g_m[idx] = gm[0];
    io.g_m[ld + idx] = gm[1];
    io.g_w0[idx] = lam[0];
#pragma unroll
    for (int c = 0; c < 6; ++c) io.g_S0[c * ld + idx] = lam[1 + c];
#pragma unroll
    for (int c = 0; c < 3; ++c) io.g_L0[c * ld + idx] = lam[7 + c];
}

template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void adjoint_kernel(AdjIo io, AdjUni u) {
    __shared__ double s_ys[BLOCK / 64][64][64];     // y, the stage points and the step's log base
    double* ys = &s_ys[threadIdx.x / 64][0][lane_id()];
    __shared__ double s_nx[BLOCK / 64][11][64];     // state and step size of the step reversed next
    double* nx = &s_nx[threadIdx.x / 64][0][lane_id()];
    const int64_t j = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (j >= u.n) return;
    const int64_t idx = io.order ? (int64_t)io.order[j] : j;
    if (idx < 0 || idx >= u.n) return;      // not a permutation entry: nothing to do
    adjoint_one(io, u, idx, io.ws + j, ys, nx);
}

// ---------------------------------------------------------------------------
// Replay of a recorded step sequence (no error control): the map whose
// discrete adjoint pn_integrate_adjoint computes, evaluated at any initial
// state.  One inspiral per lane.
// ---------------------------------------------------------------------------
struct ReplayIo {
    const double* __restrict__ m;
    const double* __restrict__ S0;
    const double* __restrict__ L0;
    const double* __restrict__ w0;
    const int32_t* __restrict__ status; // [ld] of the recorded run, or null (all OK)
    double* __restrict__ y;             // [10][ld]
    double* __restrict__ t;             // [ld]
};

// the stage derivative as stage_deriv, and the rate of t along the variable
// of the step (1 in a time step, dt/domega = 1/f_0 in an omega-step)
__device__ __forceinline__ double stage_deriv_t(const Row& R, const TermConsts& tc, const LogBase& lb,
                                                const double* Y, double* k, bool om) {
    rhs<Row, true>(R, tc, lb, Y, k);
    if (!om) return 1.0;
    const double s = 1.0 / k[0];
#pragma unroll
    for (int c = 1; c < 10; ++c) k[c] *= s;
    k[0] = 1.0;
    return s;
}

// one replayed step with t: y <- y + h sum b_i k_i, t <- t + h sum b_i r_i
__device__ __forceinline__ void replay_step_t(const Row& R, const TermConsts& tc, double* y, double& t, double h,
                                              bool om) {
    double k1[10], k2[10], k3[10], k4[10], k5[10], k6[10], Y[10];
    const LogBase lb = log_base(R, y);
    const double r1 = stage_deriv_t(R, tc, lb, y, k1, om);
#pragma unroll
    for (int c = 0; c < 10; ++c) Y[c] = __builtin_fma(h * A21, k1[c], y[c]);
    stage_deriv_t(R, tc, lb, Y, k2, om);
#pragma unroll
    for (int c = 0; c < 10; ++c) Y[c] = __builtin_fma(h * A32, k2[c], __builtin_fma(h * A31, k1[c], y[c]));
    const double r3 = stage_deriv_t(R, tc, lb, Y, k3, om);
#pragma unroll
    for (int c = 0; c < 10; ++c)
        Y[c] = __builtin_fma(h * A43, k3[c], __builtin_fma(h * A42, k2[c], __builtin_fma(h * A41, k1[c], y[c])));
    const double r4 = stage_deriv_t(R, tc, lb, Y, k4, om);
#pragma unroll
    for (int c = 0; c < 10; ++c)
        Y[c] = __builtin_fma(h * A54, k4[c], __builtin_fma(h * A53, k3[c],
               __builtin_fma(h * A52, k2[c], __builtin_fma(h * A51, k1[c], y[c]))));
    const double r5 = stage_deriv_t(R, tc, lb, Y, k5, om);
#pragma unroll
    for (int c = 0; c < 10; ++c)
        Y[c] = __builtin_fma(h * A65, k5[c], __builtin_fma(h * A64, k4[c], __builtin_fma(h * A63, k3[c],
               __builtin_fma(h * A62, k2[c], __builtin_fma(h * A61, k1[c], y[c])))));
    const double r6 = stage_deriv_t(R, tc, lb, Y, k6, om);
#pragma unroll
    for (int c = 0; c < 10; ++c)
        y[c] = __builtin_fma(h * B6, k6[c], __builtin_fma(h * B5, k5[c], __builtin_fma(h * B4, k4[c],
               __builtin_fma(h * B3, k3[c], __builtin_fma(h * B1, k1[c], y[c])))));
    t = __builtin_fma(h, B1 * r1 + B3 * r3 + B4 * r4 + B5 * r5 + B6 * r6, t);
}

template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void replay_kernel(ReplayIo io, AdjUni u) {
    const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (i >= u.n) return;
    const int64_t ld = u.ld;
    const double* tp = u.tape + i * u.tape_stride;
    const double m1 = io.m[i], m2 = io.m[ld + i];
    double y[10];
    y[0] = io.w0[i];
#pragma unroll
    for (int c = 0; c < 6; ++c) y[1 + c] = io.S0[c * ld + i];
#pragma unroll
    for (int c = 0; c < 3; ++c) y[7 + c] = io.L0[c * ld + i];
    double t = 0.0;
    // a recorded run that ended at once keeps its initial state; any other
    // recorded failure, a row that does not hold the counts of a recorded
    // run (non-integer, negative, or more steps than the tape holds), or
    // inputs the integrator refuses: NaN outputs (the tape is not read
    // beyond its counts)
    const int st = io.status ? io.status[i] : PN_ST_OK;
    const double tnt = tp[0], tnw = tp[1];
    bool ok = st == PN_ST_OK || st == PN_ST_DONE_AT_START;
    if (st == PN_ST_OK)
        ok = tnt >= 0.0 && tnw >= 0.0 && tnt + tnw <= (double)u.tape_cap && tnt == __builtin_floor(tnt) &&
             tnw == __builtin_floor(tnw);
    ok = ok && m1 > 0.0 && m2 > 0.0 && y[0] > 0.0 && finite(m1) && finite(m2);
#pragma unroll
    for (int c = 0; c < 10; ++c) ok = ok && finite(y[c]);
    if (ok && st == PN_ST_OK) {
        Row R;
        make_row(R, m1, m2, u.terms, u.theta_literal);
        const int nt = (int)tnt;
        const int N = nt + (int)tnw;
        const double* hs = tp + 2;
        for (int k = 0; k < N; ++k) {
            const bool om = k >= nt;
            const double h = (om && k == N - 1) ? u.omega_f - y[0] : hs[k];
            replay_step_t(R, u.tc, y, t, h, om);
        }
        if (N > nt) y[0] = u.omega_f;      // the run ends on omega_f exactly
    } else if (!ok) {
#pragma unroll
        for (int c = 0; c < 10; ++c) y[c] = __builtin_nan("");
        t = __builtin_nan("");
    }
#pragma unroll
    for (int c = 0; c < 10; ++c) io.y[c * ld + i] = y[c];
    io.t[i] = t;
}

// Zeroes the work counter of a persistent launch and writes its launch
// descriptor into the call's slot (one word per thread).
__global__ void prepare_launch(unsigned long long* slot, LaunchDesc desc) {
    const unsigned t = threadIdx.x;
    if (t == 0) slot[0] = 0ull;
    const unsigned long long* src = reinterpret_cast<const unsigned long long*>(&desc);
    if (t < sizeof(LaunchDesc) / 8) slot[kDescOffset + t] = src[t];
}

__global__ void rhs_kernel(int64_t n, int64_t ld, const double* __restrict__ m, const double* __restrict__ y,
                           double* __restrict__ d, int terms, int theta_literal, TermConsts tc) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    Row r;
    make_row(r, m[i], m[ld + i], terms, theta_literal);
    double yy[10], dd[10];
#pragma unroll
    for (int c = 0; c < 10; ++c) yy[c] = y[c * ld + i];
    LogBase lb;
    rhs<Row, false>(r, tc, lb, yy, dd);
#pragma unroll
    for (int c = 0; c < 10; ++c) d[c * ld + i] = dd[c];
}

__global__ void observables_kernel(int64_t n, int64_t ld, const double* __restrict__ y, double* __restrict__ dots) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double v[10];
#pragma unroll
    for (int c = 0; c < 10; ++c) v[c] = y[c * ld + i];
    const double n1 = __builtin_sqrt(v[1] * v[1] + v[2] * v[2] + v[3] * v[3]);
    const double n2 = __builtin_sqrt(v[4] * v[4] + v[5] * v[5] + v[6] * v[6]);
    const double nl = __builtin_sqrt(v[7] * v[7] + v[8] * v[8] + v[9] * v[9]);
    const double s12 = v[1] * v[4] + v[2] * v[5] + v[3] * v[6];
    const double s1l = v[1] * v[7] + v[2] * v[8] + v[3] * v[9];
    const double s2l = v[4] * v[7] + v[5] * v[8] + v[6] * v[9];
    dots[i] = (n1 > 0.0 && n2 > 0.0) ? s12 / (n1 * n2) : 0.0;
    dots[ld + i] = (n1 > 0.0 && nl > 0.0) ? s1l / (n1 * nl) : 0.0;
    dots[2 * ld + i] = (n2 > 0.0 && nl > 0.0) ? s2l / (n2 * nl) : 0.0;
}

// ---------------------------------------------------------------------------
// Host side: per-device context, argument checks, launches
// ---------------------------------------------------------------------------

// The HIP side of the call-slot bookkeeping (pn_slots.hpp).
struct HipSlotOps {
    using Stream = hipStream_t;
    using Event = hipEvent_t;
    int capturing(Stream s, bool* cap) {
        hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing(s, &st) != hipSuccess) return PN_EHIP;
        *cap = st != hipStreamCaptureStatusNone;
        return 0;
    }
    int create(Event* e) { return hipEventCreateWithFlags(e, hipEventDisableTiming) == hipSuccess ? 0 : PN_EHIP; }
    int wait(Stream s, Event e) { return hipStreamWaitEvent(s, e, 0) == hipSuccess ? 0 : PN_EHIP; }
    int record(Event e, Stream s) { return hipEventRecord(e, s) == hipSuccess ? 0 : PN_EHIP; }
    int destroy(Event e) { return hipEventDestroy(e) == hipSuccess ? 0 : PN_EHIP; }
};

// call slots: 1024 taken in turn by direct calls, 4096 for captured calls
using Slots = SlotTable<HipSlotOps, 1024, 4096>;
constexpr int kCounterSlots = Slots::kRing + Slots::kCapture;

struct DevCtx {
    std::atomic<bool> ready{false};
    int cus = 0;
    unsigned long long* counters = nullptr;   // kCounterSlots slots: work counter, launch descriptor
    Slots slots;
};

constexpr int kMaxDevices = 64;
DevCtx g_ctx[kMaxDevices];
std::mutex g_ctx_mu;

int get_ctx(DevCtx** out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return PN_ENODEV;
    DevCtx& c = g_ctx[dev];
    if (!c.ready.load(std::memory_order_acquire)) {
        std::lock_guard<std::mutex> lk(g_ctx_mu);
        if (!c.ready.load(std::memory_order_relaxed)) {
            hipDeviceProp_t prop;
            if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return PN_ENODEV;
            if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return PN_ENODEV;
            c.cus = prop.multiProcessorCount;
            void* p = nullptr;
            if (hipMalloc(&p, sizeof(unsigned long long) * kCounterSlots * kSlotWords) != hipSuccess)
                return PN_ENOMEM;
            c.counters = (unsigned long long*)p;
            c.ready.store(true, std::memory_order_release);
        }
    }
    *out = &c;
    return PN_OK;
}

// pn_integrate_noalloc: the call slot of its persistent launches (work
// counter and launch descriptor, 512 B) is this file-scope device array, so
// that the call allocates nothing.  Each device holds its own copy; host code
// uses the address hipGetSymbolAddress returns for the current device, never
// the array's name.  Every such call on a device shares the array: calls that
// overlap on one device race.
constexpr int kScratchWords = kSlotWords;
static __device__ __align__(256) unsigned long long scratch[kScratchWords];

struct ScratchDev {
    std::atomic<bool> ready{false};
    unsigned long long* ptr = nullptr;   // device address of `scratch` on this device
    int cus = 0;
};
ScratchDev g_scratch[kMaxDevices];

// Once per device, with that device current: its address of `scratch` and
// its compute-unit count (no allocation).
int get_scratch(ScratchDev** out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return PN_ENODEV;
    ScratchDev& d = g_scratch[dev];
    if (!d.ready.load(std::memory_order_acquire)) {
        std::lock_guard<std::mutex> lk(g_ctx_mu);
        if (!d.ready.load(std::memory_order_relaxed)) {
            hipDeviceProp_t prop;
            if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return PN_ENODEV;
            if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return PN_ENODEV;
            void* p = nullptr;
            if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || p == nullptr) return PN_EHIP;
            d.ptr = static_cast<unsigned long long*>(p);
            d.cus = prop.multiProcessorCount;
            d.ready.store(true, std::memory_order_release);
        }
    }
    *out = &d;
    return PN_OK;
}

int release_ctx() {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return PN_ENODEV;
    std::lock_guard<std::mutex> lk(g_ctx_mu);
    DevCtx& c = g_ctx[dev];
    if (!c.ready.load(std::memory_order_relaxed)) return PN_OK;
    c.ready.store(false, std::memory_order_release);
    HipSlotOps ops;
    const int re = c.slots.reset(ops);
    const hipError_t e = hipFree(c.counters);
    c.counters = nullptr;
    return (e == hipSuccess && re == 0) ? PN_OK : PN_EHIP;
}

TermConsts term_consts(int terms) {
    TermConsts tc;
    const bool pn_on = (terms & PN_TERM_PN) != 0;
    tc.c3 = pn_on ? 4.0 * PN_PI : 0.0;
    tc.c6lnv = pn_on ? -(1712.0 / 315.0) : 0.0;
    return tc;
}

template <int BLOCK>
hipError_t launch_static(const Io& io, const Uni& u, int precision, hipStream_t s) {
    const bool f32 = precision == PN_PREC_FP32_SPLIT;
    const bool f32x = precision == PN_PREC_FP32_STATE;
    const bool ph = io.phase != nullptr;
    const int64_t grid = (u.n + BLOCK - 1) / BLOCK;
    if (ph && f32x) hipLaunchKernelGGL(integrate_static_f32x_phase<BLOCK>, dim3((unsigned)grid), dim3(BLOCK), 0, s, io, u);
    else if (f32x) hipLaunchKernelGGL(integrate_static_f32x<BLOCK>, dim3((unsigned)grid), dim3(BLOCK), 0, s, io, u);
    else if (ph && f32) hipLaunchKernelGGL(integrate_static_f32s_phase<BLOCK>, dim3((unsigned)grid), dim3(BLOCK), 0, s, io, u);
    else if (ph) hipLaunchKernelGGL(integrate_static_f64_phase<BLOCK>, dim3((unsigned)grid), dim3(BLOCK), 0, s, io, u);
    else if (f32) hipLaunchKernelGGL(integrate_static_f32s<BLOCK>, dim3((unsigned)grid), dim3(BLOCK), 0, s, io, u);
    else if (u.tape) hipLaunchKernelGGL((integrate_static_f64<BLOCK, true>), dim3((unsigned)grid), dim3(BLOCK), 0, s, io, u);
    else hipLaunchKernelGGL((integrate_static_f64<BLOCK, false>), dim3((unsigned)grid), dim3(BLOCK), 0, s, io, u);
    return hipGetLastError();
}

// The persistent launch on the call slot `counter`: prepare_launch zeroes the
// slot's work counter and writes the descriptor, then the persistent grid.
template <int BLOCK>
hipError_t launch_persistent(const Io& io, const Uni& u, int precision, int waves_per_simd, int cus,
                             unsigned long long* counter, hipStream_t s) {
    const bool f32 = precision == PN_PREC_FP32_SPLIT;
    const bool f32x = precision == PN_PREC_FP32_STATE;
    const bool ph = io.phase != nullptr;
    LaunchDesc desc;
    desc.io = io;
    desc.u = u;
    hipLaunchKernelGGL(prepare_launch, dim3(1), dim3(64), 0, s, counter, desc);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t waves_needed = (u.n + 63) / 64;
    int64_t waves = (int64_t)cus * 4 * waves_per_simd;
    if (waves > waves_needed) waves = waves_needed;
    const int64_t grid = (waves * 64 + BLOCK - 1) / BLOCK;
    const bool gen = u.fixed || u.tend;    // not the plain adaptive run to omega_f
    const dim3 g((unsigned)grid), b(BLOCK);
    if (ph && f32x)
        hipLaunchKernelGGL(integrate_persistent_f32x_phase<BLOCK>, g, b, 0, s, u, counter);
    else if (f32x && gen)
        hipLaunchKernelGGL(integrate_persistent_f32x_modes<BLOCK>, g, b, 0, s, u, counter);
    else if (f32x)
        hipLaunchKernelGGL(integrate_persistent_f32x<BLOCK>, g, b, 0, s, u, counter);
    else if (ph && f32)
        hipLaunchKernelGGL(integrate_persistent_f32s_phase<BLOCK>, g, b, 0, s, u, counter);
    else if (ph)
        hipLaunchKernelGGL(integrate_persistent_f64_phase<BLOCK>, g, b, 0, s, u, counter);
    else if (f32 && gen)
        hipLaunchKernelGGL(integrate_persistent_f32s_modes<BLOCK>, g, b, 0, s, u, counter);
    else if (f32)
        hipLaunchKernelGGL(integrate_persistent_f32s<BLOCK>, g, b, 0, s, u, counter);
    else if (u.tape && gen)
        hipLaunchKernelGGL((integrate_persistent_f64_modes<BLOCK, true>), g, b, 0, s, u, counter);
    else if (u.tape)
        hipLaunchKernelGGL((integrate_persistent_f64<BLOCK, true>), g, b, 0, s, u, counter);
    else if (gen)
        hipLaunchKernelGGL((integrate_persistent_f64_modes<BLOCK, false>), g, b, 0, s, u, counter);
    else
        hipLaunchKernelGGL((integrate_persistent_f64<BLOCK, false>), g, b, 0, s, u, counter);
    return hipGetLastError();
}

int device_ready() {
    DevCtx* ctx = nullptr;
    return get_ctx(&ctx);
}

}  // namespace pn

using namespace pn;

extern "C" {

const char* pn_strerror(int code) {
    switch (code) {
        case PN_OK: return "PN_OK: success";
        case PN_EINVAL: return "PN_EINVAL: invalid argument";
        case PN_ENODEV: return "PN_ENODEV: no usable gfx950 device is current";
        case PN_EHIP: return "PN_EHIP: a HIP runtime call or kernel launch failed";
        case PN_ENOMEM: return "PN_ENOMEM: device context allocation failed";
        case PN_EBUSY: return "PN_EBUSY: every call slot for launches captured into graphs is taken (pn_shutdown frees them)";
        default: return "unknown pn error code";
    }
}

const char* pn_version(void) { return "pn-gfx950 0.2"; }

int pn_shutdown(void) { return release_ctx(); }

static int integrate_impl(int64_t n, int64_t ld, const double* m, const double* S0, const double* L0,
                          const double* omega0, double omega_f, double tol, const pn_opts* opt,
                          double* y_final, double* t_final, int32_t* steps, int32_t* status, double* dots,
                          double* tape, int64_t cap_steps, int32_t ckpt_every, double* phase, void* stream,
                          bool noalloc = false) {
    pn_opts o;
    std::memset(&o, 0, sizeof(o));
    if (opt) o = *opt;
    if (n < 0 || ld < n || ld > PN_MAX_N) return PN_EINVAL;
    if (n > 0 && (!m || !S0 || !L0 || !omega0 || !y_final || !t_final || !steps || !status)) return PN_EINVAL;
    const bool fixed = o.h_fixed > 0.0;
    const bool tend = o.t_end > 0.0;
    if (o.h_fixed < 0.0 || !(o.h_fixed == o.h_fixed) || !(o.t_end == o.t_end) || o.t_end < 0.0) return PN_EINVAL;
    if (fixed && !(o.h_fixed < 1e300)) return PN_EINVAL;
    if (!fixed && !(tol > 0.0 && tol < 1e300)) return PN_EINVAL;
    if (!tend && !(omega_f > 0.0 && omega_f < 1e300)) return PN_EINVAL;
    if (tend && !(o.t_end < 1e300)) return PN_EINVAL;
    if (!(o.h0 == o.h0) || o.h0 >= 1e300) return PN_EINVAL;
    if (o.schedule != PN_SCHED_PERSISTENT && o.schedule != PN_SCHED_STATIC) return PN_EINVAL;
    if (o.precision != PN_PREC_FP64 && o.precision != PN_PREC_FP32_SPLIT && o.precision != PN_PREC_FP32_STATE)
        return PN_EINVAL;
    const int block = o.block ? o.block : 256;
    if (block != 64 && block != 128 && block != 256 && block != 512) return PN_EINVAL;
    const int wps = o.waves_per_simd ? o.waves_per_simd
                                     : (o.precision == PN_PREC_FP32_SPLIT ? kWpeF32
                                        : o.precision == PN_PREC_FP32_STATE ? kWpeF32S : kWpeF64);
    if (wps < 1 || wps > 8) return PN_EINVAL;
    const int refill = o.refill_min ? o.refill_min : 4;
    if (refill < 1 || refill > 64) return PN_EINVAL;
    if (o.terms < 0 || o.terms > PN_TERM_ALL) return PN_EINVAL;
    if (o.theta_literal != 0 && o.theta_literal != 1) return PN_EINVAL;
    if (o.order && n > INT32_MAX) return PN_EINVAL;
    if (((uintptr_t)o.packed & 15) != 0) return PN_EINVAL;
    if (tape) {
        if (o.precision != PN_PREC_FP64 || tend) return PN_EINVAL;
        if (cap_steps < 1 || cap_steps > (1 << 28) || ckpt_every < 1 || ckpt_every > 4096) return PN_EINVAL;
    }
    if (n == 0) return PN_OK;

    DevCtx* ctx = nullptr;
    ScratchDev* sd = nullptr;
    const int rc = noalloc ? get_scratch(&sd) : get_ctx(&ctx);
    if (rc != PN_OK) return rc;

    Uni u;
    u.omega_f = tend ? 0.0 : omega_f;
    u.tol = fixed ? 1.0 : tol;
    u.h0 = o.h0 > 0.0 ? o.h0 : 10.0;
    u.h_fixed = o.h_fixed;
    u.t_end = o.t_end;
    u.terms = o.terms > 0 ? o.terms : PN_TERM_ALL;
    u.theta_literal = o.theta_literal;
    u.tc = term_consts(u.terms);
    u.tcf.c3 = (float)u.tc.c3;
    u.tcf.c6lnv = (float)u.tc.c6lnv;
    u.n = n;
    u.ld = ld;
    u.max_steps = o.max_steps > 0 ? o.max_steps : 10000000LL;
    u.fixed = fixed;
    u.tend = tend;
    u.refill_min = refill;
    u.rr_on = (u.terms & PN_TERM_RR) != 0;
    u.tape = tape;
    u.tape_stride = tape ? (int64_t)pn_tape_stride(cap_steps, ckpt_every) : 0;
    u.tape_cap = (int)cap_steps;
    u.ckpt_every = ckpt_every > 0 ? ckpt_every : 1;

    Io io;
    io.m = m; io.S0 = S0; io.L0 = L0; io.w0 = omega0;
    io.y = y_final; io.t = t_final; io.steps = steps; io.status = status; io.dots = dots;
    io.phase = phase;
    io.order = o.order;
    io.packed = o.packed;

    hipStream_t s = (hipStream_t)stream;
    if (o.schedule == PN_SCHED_STATIC) {
        hipError_t e;
        switch (block) {
            case 64: e = launch_static<64>(io, u, o.precision, s); break;
            case 128: e = launch_static<128>(io, u, o.precision, s); break;
            case 512: e = launch_static<512>(io, u, o.precision, s); break;
            default: e = launch_static<256>(io, u, o.precision, s); break;
        }
        return e == hipSuccess ? PN_OK : PN_EHIP;
    }
    const int cus = noalloc ? sd->cus : ctx->cus;
    auto launch = [&](unsigned long long* counter) {
        hipError_t e;
        switch (block) {
            case 64: e = launch_persistent<64>(io, u, o.precision, wps, cus, counter, s); break;
            case 128: e = launch_persistent<128>(io, u, o.precision, wps, cus, counter, s); break;
            case 512: e = launch_persistent<512>(io, u, o.precision, wps, cus, counter, s); break;
            default: e = launch_persistent<256>(io, u, o.precision, wps, cus, counter, s); break;
        }
        return e == hipSuccess ? PN_OK : PN_EHIP;
    };
    if (noalloc) return launch(sd->ptr);
    HipSlotOps ops;
    return ctx->slots.run(ops, s, PN_EBUSY,
                          [&](int k) { return launch(ctx->counters + (size_t)k * kSlotWords); });
}

int pn_integrate(int64_t n, int64_t ld, const double* m, const double* S0, const double* L0,
                 const double* omega0, double omega_f, double tol, const pn_opts* opt,
                 double* y_final, double* t_final, int32_t* steps, int32_t* status, double* dots,
                 void* stream) {
    return integrate_impl(n, ld, m, S0, L0, omega0, omega_f, tol, opt, y_final, t_final, steps, status, dots,
                          nullptr, 0, 0, nullptr, stream);
}

int pn_integrate_noalloc(int64_t n, int64_t ld, const double* m, const double* S0, const double* L0,
                         const double* omega0, double omega_f, double tol, const pn_opts* opt,
                         double* y_final, double* t_final, int32_t* steps, int32_t* status, double* dots,
                         void* stream) {
    return integrate_impl(n, ld, m, S0, L0, omega0, omega_f, tol, opt, y_final, t_final, steps, status, dots,
                          nullptr, 0, 0, nullptr, stream, true);
}

int pn_integrate_phase(int64_t n, int64_t ld, const double* m, const double* S0, const double* L0,
                       const double* omega0, double omega_f, double tol, const pn_opts* opt,
                       double* y_final, double* t_final, int32_t* steps, int32_t* status, double* dots,
                       double* phase, void* stream) {
    if (n > 0 && !phase) return PN_EINVAL;
    return integrate_impl(n, ld, m, S0, L0, omega0, omega_f, tol, opt, y_final, t_final, steps, status, dots,
                          nullptr, 0, 0, phase, stream);
}

int pn_autotune(int64_t n, int64_t ld, const double* m, const double* S0, const double* L0,
                const double* omega0, double omega_f, double tol, const pn_opts* opt, int64_t sample,
                int32_t reps, double* y_final, double* t_final, int32_t* steps, int32_t* status,
                double* dots, pn_opts* best, double* times_ms, void* stream) {
    if (!best || n < 0 || ld < n || ld > PN_MAX_N) return PN_EINVAL;
    pn_opts base;
    std::memset(&base, 0, sizeof(base));
    if (opt) base = *opt;
    const int64_t ns = (sample <= 0 || sample > n) ? n : sample;
    const int r = reps > 0 ? reps : 2;
    static const int kRefill[4] = {2, 3, 4, 6};
    static const int kBlocks[2] = {128, 256};
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess) return PN_EHIP;
    if (hipEventCreate(&e1) != hipSuccess) { (void)hipEventDestroy(e0); return PN_EHIP; }
    int rc = PN_OK;
    double best_ms = 0.0;
    *best = base;
    // warm-up with the base options (also validates every argument)
    rc = pn_integrate(ns, ld, m, S0, L0, omega0, omega_f, tol, &base, y_final, t_final, steps, status, dots, stream);
    for (int c = 0; c < 8 && rc == PN_OK; ++c) {
        pn_opts o = base;
        o.refill_min = kRefill[c / 2];
        o.block = kBlocks[c % 2];
        if (hipEventRecord(e0, s) != hipSuccess) { rc = PN_EHIP; break; }
        for (int k = 0; k < r && rc == PN_OK; ++k)
            rc = pn_integrate(ns, ld, m, S0, L0, omega0, omega_f, tol, &o, y_final, t_final, steps, status, dots,
                              stream);
        if (rc != PN_OK) break;
        float ms = 0.0f;
        if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
            rc = PN_EHIP;
            break;
        }
        const double mean = (double)ms / r;
        if (times_ms) times_ms[c] = mean;
        if (c == 0 || mean < best_ms) {
            best_ms = mean;
            *best = o;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return rc;
}

size_t pn_tape_stride(int64_t cap_steps, int32_t ckpt_every) {
    if (cap_steps < 1 || ckpt_every < 1) return 0;
    return (size_t)(2 + cap_steps + 10 * (cap_steps / ckpt_every + 1));
}

int pn_integrate_record(int64_t n, int64_t ld, const double* m, const double* S0, const double* L0,
                        const double* omega0, double omega_f, double tol, const pn_opts* opt,
                        double* y_final, double* t_final, int32_t* steps, int32_t* status, double* dots,
                        double* tape, int64_t cap_steps, int32_t ckpt_every, void* stream) {
    if (n > 0 && !tape) return PN_EINVAL;
    return integrate_impl(n, ld, m, S0, L0, omega0, omega_f, tol, opt, y_final, t_final, steps, status, dots,
                          tape, cap_steps, ckpt_every, nullptr, stream);
}

size_t pn_adjoint_workspace_bytes(int64_t n, int32_t ckpt_every) {
    if (n < 0 || n > PN_MAX_N || ckpt_every < 1) return 0;
    // the replayed states and step sizes of one segment per inspiral
    return (size_t)n * (size_t)ckpt_every * 11 * sizeof(double);
}

int pn_integrate_adjoint(int64_t n, int64_t ld, const double* m, double omega_f, const pn_opts* opt,
                         const double* tape, int64_t cap_steps, int32_t ckpt_every, const int32_t* status,
                         const double* gy_final, const double* gt_final, double* g_m, double* g_S0,
                         double* g_L0, double* g_omega0, double* workspace, size_t ws_bytes,
                         const int32_t* order, void* stream) {
    if (n < 0 || ld < n || ld > PN_MAX_N) return PN_EINVAL;
    if (cap_steps < 1 || cap_steps > (1 << 28) || ckpt_every < 1 || ckpt_every > 4096) return PN_EINVAL;
    if (n > 0 && (!m || !tape || !status || !gy_final || !g_m || !g_S0 || !g_L0 || !g_omega0 || !workspace))
        return PN_EINVAL;
    if (!(omega_f > 0.0 && omega_f < 1e300)) return PN_EINVAL;
    if (ws_bytes < pn_adjoint_workspace_bytes(n, ckpt_every)) return PN_EINVAL;
    const int terms = (opt && opt->terms > 0) ? opt->terms : PN_TERM_ALL;
    const int lit = opt ? opt->theta_literal : 0;
    if ((opt && opt->terms > PN_TERM_ALL) || (lit != 0 && lit != 1)) return PN_EINVAL;
    if (opt && (opt->precision != PN_PREC_FP64 || opt->t_end > 0.0 || opt->h_fixed > 0.0)) return PN_EINVAL;
    if (n == 0) return PN_OK;
    DevCtx* ctx = nullptr;
    int rc = get_ctx(&ctx);
    if (rc != PN_OK) return rc;
    AdjUni u;
    u.omega_f = omega_f;
    u.tc = term_consts(terms);
    u.n = n;
    u.ld = ld;
    u.terms = terms;
    u.theta_literal = lit;
    u.tape = tape;
    u.tape_stride = (int64_t)pn_tape_stride(cap_steps, ckpt_every);
    u.tape_cap = (int)cap_steps;
    u.ckpt_every = ckpt_every;
    AdjIo io;
    io.m = m; io.status = status; io.gy = gy_final; io.gt = gt_final;
    io.g_m = g_m; io.g_S0 = g_S0; io.g_L0 = g_L0; io.g_w0 = g_omega0; io.order = order;
    io.ws = workspace;                                       // [K][11][n] replayed states and steps
    const int64_t grid = (n + 127) / 128;
    hipLaunchKernelGGL(adjoint_kernel<128>, dim3((unsigned)grid), dim3(128), 0, (hipStream_t)stream, io, u);
    return hipGetLastError() == hipSuccess ? PN_OK : PN_EHIP;
}

size_t pn_ckpt_bytes(int64_t n, int64_t cap_steps, int32_t ckpt_every) {
    if (n < 0 || n > PN_MAX_N || cap_steps < 1 || cap_steps > (1 << 28) || ckpt_every < 1 || ckpt_every > 4096)
        return 0;
    return (size_t)n * pn_tape_stride(cap_steps, ckpt_every) * sizeof(double);
}

int pn_integrate_replay(int64_t n, int64_t ld, const double* m, const double* S0, const double* L0,
                        const double* omega0, double omega_f, const pn_opts* opt, const double* tape,
                        int64_t cap_steps, int32_t ckpt_every, const int32_t* status, double* y_final,
                        double* t_final, void* stream) {
    if (n < 0 || ld < n || ld > PN_MAX_N) return PN_EINVAL;
    if (cap_steps < 1 || cap_steps > (1 << 28) || ckpt_every < 1 || ckpt_every > 4096) return PN_EINVAL;
    if (n > 0 && (!m || !S0 || !L0 || !omega0 || !tape || !y_final || !t_final)) return PN_EINVAL;
    if (!(omega_f > 0.0 && omega_f < 1e300)) return PN_EINVAL;
    const int terms = (opt && opt->terms > 0) ? opt->terms : PN_TERM_ALL;
    const int lit = opt ? opt->theta_literal : 0;
    if ((opt && opt->terms > PN_TERM_ALL) || (lit != 0 && lit != 1)) return PN_EINVAL;
    if (opt && (opt->precision != PN_PREC_FP64 || opt->t_end > 0.0 || opt->h_fixed > 0.0)) return PN_EINVAL;
    if (n == 0) return PN_OK;
    AdjUni u{};
    u.omega_f = omega_f;
    u.tc = term_consts(terms);
    u.n = n;
    u.ld = ld;
    u.terms = terms;
    u.theta_literal = lit;
    u.tape = tape;
    u.tape_stride = (int64_t)pn_tape_stride(cap_steps, ckpt_every);
    u.tape_cap = (int)cap_steps;
    u.ckpt_every = ckpt_every;
    ReplayIo io;
    io.m = m; io.S0 = S0; io.L0 = L0; io.w0 = omega0; io.status = status; io.y = y_final; io.t = t_final;
    const int64_t grid = (n + 127) / 128;
    hipLaunchKernelGGL(replay_kernel<128>, dim3((unsigned)grid), dim3(128), 0, (hipStream_t)stream, io, u);
    return hipGetLastError() == hipSuccess ? PN_OK : PN_EHIP;
}

int pn_rhs(int64_t n, int64_t ld, const double* m, const double* y, double* dydt, const pn_opts* opt,
           void* stream) {
    if (n < 0 || ld < n || ld > PN_MAX_N) return PN_EINVAL;
    if (n > 0 && (!m || !y || !dydt)) return PN_EINVAL;
    const int terms = (opt && opt->terms > 0) ? opt->terms : PN_TERM_ALL;
    const int lit = opt ? opt->theta_literal : 0;
    if ((opt && opt->terms > PN_TERM_ALL) || (lit != 0 && lit != 1)) return PN_EINVAL;
    if (n == 0) return PN_OK;
    DevCtx* ctx = nullptr;
    int rc = get_ctx(&ctx);
    if (rc != PN_OK) return rc;
    const int64_t grid = (n + 255) / 256;
    hipLaunchKernelGGL(rhs_kernel, dim3((unsigned)grid), dim3(256), 0, (hipStream_t)stream, n, ld, m, y,
                       dydt, terms, lit, term_consts(terms));
    return hipGetLastError() == hipSuccess ? PN_OK : PN_EHIP;
}

int pn_observables(int64_t n, int64_t ld, const double* y, double* dots, void* stream) {
    if (n < 0 || ld < n || ld > PN_MAX_N) return PN_EINVAL;
    if (n > 0 && (!y || !dots)) return PN_EINVAL;
    if (n == 0) return PN_OK;
    DevCtx* ctx = nullptr;
    int rc = get_ctx(&ctx);
    if (rc != PN_OK) return rc;
    const int64_t grid = (n + 255) / 256;
    hipLaunchKernelGGL(observables_kernel, dim3((unsigned)grid), dim3(256), 0, (hipStream_t)stream, n, ld, y,
                       dots);
    return hipGetLastError() == hipSuccess ? PN_OK : PN_EHIP;
}

}  // extern "C"
