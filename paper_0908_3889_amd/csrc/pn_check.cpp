// pn_check.cpp -- the check of GPU results against the CPU on a subset
// (Sec. III: kernels on the GPU fail without reporting it, so the paper ran
// the same inspirals on the CPU for part of each population and compared).
//
// A host integrator of the same method as the GPU kernels (Eqs. (1)-(4),
// adaptive Dormand-Prince with the same error norm, step control and final
// stretch in omega), in plain FP64 C++ with the library's cube root and log
// replaced by the C library's: its results agree with the kernels' to
// rounding, so accepted and rejected step counts agree except where a step's
// error norm lies within rounding of the acceptance threshold.
// pn_check_start runs it on host threads over a sample while the GPU
// integrates; pn_check_finish compares the GPU's outputs for the sample and
// flags the inspirals that disagree.
#include <sched.h>

#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <thread>
#include <vector>

#include "pn.h"

namespace pn_host {

// Dormand-Prince RK5(4)7M (Dormand & Prince 1980): nodes' rows a_sj, the
// 5th-order weights b_j (= the 7th stage's row, FSAL) and e_j = b_j - bhat_j
constexpr double A21 = 1.0 / 5.0;
constexpr double A31 = 3.0 / 40.0, A32 = 9.0 / 40.0;
constexpr double A41 = 44.0 / 45.0, A42 = -56.0 / 15.0, A43 = 32.0 / 9.0;
constexpr double A51 = 19372.0 / 6561.0, A52 = -25360.0 / 2187.0, A53 = 64448.0 / 6561.0, A54 = -212.0 / 729.0;
constexpr double A61 = 9017.0 / 3168.0, A62 = -355.0 / 33.0, A63 = 46732.0 / 5247.0, A64 = 49.0 / 176.0,
                 A65 = -5103.0 / 18656.0;
constexpr double B1 = 35.0 / 384.0, B3 = 500.0 / 1113.0, B4 = 125.0 / 192.0, B5 = -2187.0 / 6784.0,
                 B6 = 11.0 / 84.0;
constexpr double E1 = 71.0 / 57600.0, E3 = -71.0 / 16695.0, E4 = 71.0 / 1920.0, E5 = -17253.0 / 339200.0,
                 E6 = 22.0 / 525.0, E7 = -1.0 / 40.0;
constexpr double kPi = 3.14159265358979323846;
constexpr double kGammaE = 0.57721566490153286061;

struct Coeffs {          // the per-inspiral constants of Eqs. (1)-(4)
    double M, c2, so1, so2, c4, ssd, c5, c6, c7, K, g1, g2, sigm, lam;
    double c3, c6lnv;    // 4 pi and -1712/315 when the PN terms are on
};

Coeffs coeffs(double m1, double m2, int terms, int theta_literal) {
    Coeffs c;
    const double M = m1 + m2, eta = m1 * m2 / (M * M);
    const bool pn = terms & PN_TERM_PN;
    const double fso = (terms & PN_TERM_SO_WDOT) ? 1.0 : 0.0, fss = (terms & PN_TERM_SS_WDOT) ? 1.0 : 0.0;
    c.M = M;
    c.c2 = pn ? -(743.0 + 924.0 * eta) / 336.0 : 0.0;
    c.so1 = fso * (113.0 * (m1 / M) * (m1 / M) + 75.0 * eta) / (12.0 * m1 * m1);
    c.so2 = fso * (113.0 * (m2 / M) * (m2 / M) + 75.0 * eta) / (12.0 * m2 * m2);
    c.c4 = pn ? 34103.0 / 18144.0 + 13661.0 / 2016.0 * eta + 59.0 / 18.0 * eta * eta : 0.0;
    c.ssd = fss * eta / (48.0 * m1 * m1 * m2 * m2);
    c.c5 = pn ? -(4159.0 + 15876.0 * eta) * kPi / 672.0 : 0.0;
    // 3PN constant with ln(16 x^2) split into ln 16 + 2 ln x; theta_hat =
    // 1039/4620 multiplies eta once, or eta^2 as printed with theta_literal
    const double theta = (88.0 / 3.0) * (1039.0 / 4620.0) * (theta_literal ? eta : 1.0);
    c.c6 = pn ? 16447322263.0 / 139708800.0 - 1712.0 / 105.0 * kGammaE + 16.0 / 3.0 * kPi * kPi +
                    (-273811877.0 / 1088640.0 + 451.0 / 48.0 * kPi * kPi - theta) * eta + 541.0 / 896.0 * eta * eta -
                    5605.0 / 2592.0 * eta * eta * eta - 856.0 / 105.0 * std::log(16.0)
              : 0.0;
    c.c7 = pn ? (-4415.0 / 4032.0 + 358675.0 / 6048.0 * eta + 91495.0 / 1512.0 * eta * eta) * kPi : 0.0;
    c.K = (terms & PN_TERM_RR) ? 96.0 / 5.0 * eta : 0.0;
    c.g1 = (terms & PN_TERM_SO_PREC) ? eta * (4.0 + 3.0 * m2 / m1) : 0.0;
    c.g2 = (terms & PN_TERM_SO_PREC) ? eta * (4.0 + 3.0 * m1 / m2) : 0.0;
    c.sigm = (terms & PN_TERM_SS_PREC) ? 1.0 / M : 0.0;
    c.lam = 1.0 / (eta * M * M);
    c.c3 = pn ? 4.0 * kPi : 0.0;
    c.c6lnv = pn ? -1712.0 / 315.0 : 0.0;
    return c;
}

// dy/dt of Eqs. (1)-(4) at y = (omega, S1, S2, L_hat), x = (M omega)^{1/3}
void rhs(const Coeffs& c, const double* y, double* d) {
    const double w = y[0], v = c.M * w;
    const double x = std::cbrt(v), lnv = std::log(std::fabs(v)), x2 = x * x;
    const double* a = y + 1;
    const double* b = y + 4;
    const double* L = y + 7;
    const double LS1 = L[0] * a[0] + L[1] * a[1] + L[2] * a[2];
    const double LS2 = L[0] * b[0] + L[1] * b[1] + L[2] * b[2];
    const double S12 = a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
    // 1 + x^2 (c2 + x (c3' + x (c4' + x (c5 + x (c6' + x c7)))))
    const double c3p = c.c3 - c.so1 * LS1 - c.so2 * LS2;
    const double c4p = c.c4 - c.ssd * (247.0 * S12 - 721.0 * LS1 * LS2);
    const double c6p = c.c6 + c.c6lnv * lnv;
    const double B = 1.0 + x2 * (c.c2 + x * (c3p + x * (c4p + x * (c.c5 + x * (c6p + x * c.c7)))));
    d[0] = c.K * w * w * x2 * v * B;                  // x^5 = x^2 v
    // Omega_1 = (w/2)[(g1 x^2 - 3 (w/M) L.S2) L + (w/M) S2], Omega_2 likewise
    const double p = 0.5 * w, sv = c.sigm * w;
    const double al1 = p * (c.g1 * x2 - 3.0 * sv * LS2), al2 = p * (c.g2 * x2 - 3.0 * sv * LS1), be = p * sv;
    double o[3], g[3];
    for (int i = 0; i < 3; ++i) {
        o[i] = al1 * L[i] + be * b[i];
        g[i] = al2 * L[i] + be * a[i];
    }
    d[1] = o[1] * a[2] - o[2] * a[1];
    d[2] = o[2] * a[0] - o[0] * a[2];
    d[3] = o[0] * a[1] - o[1] * a[0];
    d[4] = g[1] * b[2] - g[2] * b[1];
    d[5] = g[2] * b[0] - g[0] * b[2];
    d[6] = g[0] * b[1] - g[1] * b[0];
    const double q = -c.lam * x;
    for (int i = 0; i < 3; ++i) d[7 + i] = q * (d[1 + i] + d[4 + i]);
}

struct Opts {
    double omega_f, tol, h0, h_fixed, t_end;
    int64_t max_steps;
    int terms, theta_literal;
    bool fixed, tend, rr_on;
};

struct Result {
    double y[10], t;
    int acc, rej, nrhs, status;
};

// the derivative with respect to the current variable: d/dt, or d/d omega
// (the spin and L_hat rates over d omega/dt, 1 for omega); dt = dt/d(variable)
void deriv(const Coeffs& c, const double* y, bool om, double* k, double& dt) {
    rhs(c, y, k);
    dt = 1.0;
    if (om) {
        dt = 1.0 / k[0];
        for (int i = 1; i < 10; ++i) k[i] *= dt;
        k[0] = 1.0;
    }
}

Result integrate_one(double m1, double m2, const double* y0, const Opts& o) {
    Result r;
    std::memcpy(r.y, y0, sizeof(r.y));
    r.t = 0.0;
    r.acc = r.rej = r.nrhs = 0;
    bool bad = !(m1 > 0.0) || !(m2 > 0.0) || !(y0[0] > 0.0) || !std::isfinite(m1) || !std::isfinite(m2);
    for (int i = 0; i < 10; ++i) bad = bad || !std::isfinite(y0[i]);
    if (bad) { r.status = PN_ST_BAD_INPUT; return r; }
    if (!o.tend && !(y0[0] < o.omega_f)) { r.status = PN_ST_DONE_AT_START; return r; }
    const Coeffs c = coeffs(m1, m2, o.terms, o.theta_literal);
    double* y = r.y;
    double k1[10], dt1;
    deriv(c, y, false, k1, dt1);
    r.nrhs = 1;
    double h = o.fixed ? o.h_fixed : o.h0;
    bool om = false, last_rej = false;
    for (;;) {
        // outcomes known before the step, the step limit first
        if (r.acc + r.rej >= o.max_steps) { r.status = PN_ST_MAX_STEPS; return r; }
        if (om ? dt1 <= 0.0 : (o.rr_on && k1[0] <= 0.0)) { r.status = PN_ST_OMEGADOT_NONPOSITIVE; return r; }
        const double remain = om ? o.omega_f - y[0] : (o.tend ? o.t_end - r.t : 0.0);
        const bool last = (om || o.tend) && h >= remain;
        const double hs = last ? remain : h;
        double k[7][10], dt[7], Y[10];
        std::memcpy(k[0], k1, sizeof(k1));
        dt[0] = dt1;
        static const double A[6][5] = {{A21}, {A31, A32}, {A41, A42, A43}, {A51, A52, A53, A54},
                                       {A61, A62, A63, A64, A65}, {B1, 0.0, B3, B4, B5}};
        for (int s = 1; s < 7; ++s) {
            for (int i = 0; i < 10; ++i) {
                double acc = 0.0;
                for (int j = 0; j < s && j < 5; ++j) acc += A[s - 1][j] * k[j][i];
                if (s == 6) acc += B6 * k[5][i];
                Y[i] = y[i] + hs * acc;
            }
            deriv(c, Y, om, k[s], dt[s]);
        }
        r.nrhs += 6;
        // Y is the 5th-order solution (stage 7's point); error estimate and norm
        static const double E[7] = {E1, 0.0, E3, E4, E5, E6, E7};
        double z = 0.0;
        bool fin = true;
        for (int i = 0; i < 10; ++i) {
            double e = 0.0;
            for (int j = 0; j < 7; ++j) e += E[j] * k[j][i];
            e *= hs;
            const double sc = o.tol + o.tol * std::fmax(std::fabs(y[i]), std::fabs(Y[i]));
            z += (e / sc) * (e / sc);
            fin = fin && std::isfinite(Y[i]);
        }
        z *= 0.1;
        fin = fin && (o.fixed || !std::isnan(z));
        if (!fin) { r.status = PN_ST_NONFINITE; return r; }
        const bool acc = o.fixed || z <= 1.0 + 2.220446049250313e-16;
        // step factor: safety 0.9, exponent 1/5 of err = sqrt(z), clamped to
        // [0.2, 5], no growth right after a rejection
        double fac = 1.0;
        if (!o.fixed) {
            const double zc = std::fmin(std::fmax(z, 9.313225746154785e-10), 1.073741824e9);
            const double p = 0.9 * std::pow(zc, -0.1);
            const double lo = std::fmax(p, 0.2);
            fac = !acc ? lo : std::fmin(lo, last_rej ? 1.0 : 5.0);
        }
        if (acc && !om && !o.tend && Y[0] > o.omega_f) {
            // past omega_f: finish the stretch with omega as the variable
            const double s = 1.0 / k1[0];
            for (int i = 1; i < 10; ++i) k1[i] *= s;
            k1[0] = 1.0;
            dt1 = s;
            h = o.omega_f - y[0];
            last_rej = false;
            om = true;
            continue;
        }
        if (!acc) {
            ++r.rej;
            h = hs * fac;
            last_rej = true;
            const double scale = om ? std::fabs(y[0]) : std::fmax(1.0, std::fabs(r.t));
            if (h < 1e-14 * scale) { r.status = PN_ST_H_UNDERFLOW; return r; }
            continue;
        }
        double dts = 0.0;
        static const double Bw[7] = {B1, 0.0, B3, B4, B5, B6, 0.0};
        for (int j = 0; j < 7; ++j) dts += Bw[j] * dt[j];
        r.t = om ? r.t + hs * dts : r.t + hs;
        const bool done = last || (!om && !o.tend && Y[0] == o.omega_f);
        std::memcpy(y, Y, sizeof(Y));
        std::memcpy(k1, k[6], sizeof(k1));
        dt1 = dt[6];
        ++r.acc;
        if (done) {
            if (om) y[0] = o.omega_f;
            r.status = PN_ST_OK;
            return r;
        }
        if (!o.fixed) h = hs * fac;
        last_rej = false;
    }
}

Opts make_opts(double omega_f, double tol, const pn_opts* opt) {
    pn_opts p;
    std::memset(&p, 0, sizeof(p));
    if (opt) p = *opt;
    Opts o;
    o.fixed = p.h_fixed > 0.0;
    o.tend = p.t_end > 0.0;
    o.omega_f = o.tend ? 0.0 : omega_f;
    o.tol = o.fixed ? 1.0 : tol;
    o.h0 = p.h0 > 0.0 ? p.h0 : 10.0;
    o.h_fixed = p.h_fixed;
    o.t_end = p.t_end;
    o.max_steps = p.max_steps > 0 ? p.max_steps : 10000000LL;
    o.terms = p.terms > 0 ? p.terms : PN_TERM_ALL;
    o.theta_literal = p.theta_literal;
    o.rr_on = (o.terms & PN_TERM_RR) != 0;
    return o;
}

bool opts_valid(double omega_f, double tol, const pn_opts* opt) {
    pn_opts p;
    std::memset(&p, 0, sizeof(p));
    if (opt) p = *opt;
    const bool fixed = p.h_fixed > 0.0, tend = p.t_end > 0.0;
    if (p.h_fixed < 0.0 || p.h_fixed != p.h_fixed || p.t_end != p.t_end || p.t_end < 0.0) return false;
    if (fixed && !(p.h_fixed < 1e300)) return false;
    if (!fixed && !(tol > 0.0 && tol < 1e300)) return false;
    if (!tend && !(omega_f > 0.0 && omega_f < 1e300)) return false;
    if (tend && !(p.t_end < 1e300)) return false;
    if (p.terms < 0 || p.terms > PN_TERM_ALL || (p.theta_literal != 0 && p.theta_literal != 1)) return false;
    return true;
}

// host arrays of k inspirals (SoA, leading dimension ld) and their results
struct Batch {
    int64_t k = 0, ld = 0;
    std::vector<double> m, S, L, w0;
    Opts o{};
    std::vector<Result> res;
    std::atomic<int64_t> next{0};
    std::vector<std::thread> threads;
    std::chrono::steady_clock::time_point t0;
    std::atomic<int64_t> done_ns{0};
    std::atomic<int> running{0};

    void work() {
        for (;;) {
            const int64_t i = next.fetch_add(1);
            if (i >= k) break;
            double y0[10];
            y0[0] = w0[i];
            for (int c = 0; c < 6; ++c) y0[1 + c] = S[c * k + i];
            for (int c = 0; c < 3; ++c) y0[7 + c] = L[c * k + i];
            res[i] = integrate_one(m[i], m[k + i], y0, o);
        }
        if (running.fetch_sub(1) == 1) {
            const auto dt = std::chrono::steady_clock::now() - t0;
            done_ns.store(std::chrono::duration_cast<std::chrono::nanoseconds>(dt).count());
        }
    }
};

// nthreads, or (<= 0) the number of cores this process may run on
int threads_for(int32_t nthreads) {
    if (nthreads > 0) return nthreads;
    cpu_set_t set;
    CPU_ZERO(&set);
    if (sched_getaffinity(0, sizeof(set), &set) == 0) {
        const int c = CPU_COUNT(&set);
        if (c > 0) return c;
    }
    const unsigned hw = std::thread::hardware_concurrency();
    return hw > 0 ? (int)hw : 1;
}

}  // namespace pn_host

using namespace pn_host;

struct pn_check {
    Batch b;
};

extern "C" {

int pn_check_integrate_host(int64_t n, int64_t ld, const double* m, const double* S0, const double* L0,
                            const double* omega0, double omega_f, double tol, const pn_opts* opt,
                            double* y_final, double* t_final, int32_t* steps, int32_t* status,
                            int32_t nthreads) {
    if (n < 0 || ld < n || ld > PN_MAX_N) return PN_EINVAL;
    if (n == 0) return PN_OK;
    if (!m || !S0 || !L0 || !omega0 || !y_final || !t_final || !steps || !status) return PN_EINVAL;
    if (!opts_valid(omega_f, tol, opt)) return PN_EINVAL;
    const Opts o = make_opts(omega_f, tol, opt);
    std::atomic<int64_t> next{0};
    auto work = [&]() {
        for (;;) {
            const int64_t i = next.fetch_add(1);
            if (i >= n) break;
            double y0[10];
            y0[0] = omega0[i];
            for (int c = 0; c < 6; ++c) y0[1 + c] = S0[c * ld + i];
            for (int c = 0; c < 3; ++c) y0[7 + c] = L0[c * ld + i];
            const Result r = integrate_one(m[i], m[ld + i], y0, o);
            for (int c = 0; c < 10; ++c) y_final[c * ld + i] = r.y[c];
            t_final[i] = r.t;
            steps[i] = r.acc;
            steps[ld + i] = r.rej;
            steps[2 * ld + i] = r.nrhs;
            status[i] = r.status;
        }
    };
    const int nt = (int)std::min<int64_t>(threads_for(nthreads), n);
    std::vector<std::thread> pool;
    try {
        for (int i = 1; i < nt; ++i) pool.emplace_back(work);
    } catch (...) {
    }
    work();
    for (auto& t : pool) t.join();
    return PN_OK;
}

int pn_check_start(pn_check** handle, int64_t k, int64_t ld, const double* m, const double* S0, const double* L0,
                   const double* omega0, double omega_f, double tol, const pn_opts* opt, int32_t nthreads) {
    if (!handle) return PN_EINVAL;
    *handle = nullptr;
    if (k < 0 || ld < k || ld > PN_MAX_N) return PN_EINVAL;
    if (k > 0 && (!m || !S0 || !L0 || !omega0)) return PN_EINVAL;
    if (!opts_valid(omega_f, tol, opt)) return PN_EINVAL;
    pn_check* c = new (std::nothrow) pn_check;
    if (!c) return PN_ENOMEM;
    Batch& b = c->b;
    b.k = k;
    b.o = make_opts(omega_f, tol, opt);
    // the sample is copied, so the caller's arrays may change once this returns
    b.m.resize(2 * k);
    b.S.resize(6 * k);
    b.L.resize(3 * k);
    b.w0.resize(k);
    b.res.resize(k);
    for (int64_t i = 0; i < k; ++i) {
        b.w0[i] = omega0[i];
        for (int cc = 0; cc < 2; ++cc) b.m[cc * k + i] = m[cc * ld + i];
        for (int cc = 0; cc < 6; ++cc) b.S[cc * k + i] = S0[cc * ld + i];
        for (int cc = 0; cc < 3; ++cc) b.L[cc * k + i] = L0[cc * ld + i];
    }
    b.t0 = std::chrono::steady_clock::now();
    const int nt = (int)std::max<int64_t>(1, std::min<int64_t>(threads_for(nthreads), k));
    b.running.store(nt);
    try {
        for (int i = 0; i < nt; ++i) b.threads.emplace_back([&b]() { b.work(); });
    } catch (...) {
        // fewer threads than asked for: the ones started finish the sample
        b.running.fetch_sub(nt - (int)b.threads.size());
        if (b.threads.empty()) {
            delete c;
            return PN_ENOMEM;
        }
    }
    *handle = c;
    return PN_OK;
}

int pn_check_finish(pn_check* handle, const double* y_gpu, const int32_t* steps_gpu, const int32_t* status_gpu,
                    int64_t ld_gpu, double dot_tol, int32_t* flags, pn_check_report* report) {
    if (!handle) return PN_EINVAL;
    Batch& b = handle->b;
    for (auto& t : b.threads) t.join();
    b.threads.clear();
    int rc = PN_OK;
    const int64_t k = b.k;
    if (ld_gpu < k || (k > 0 && (!y_gpu || !steps_gpu || !status_gpu)) || !(dot_tol >= 0.0)) rc = PN_EINVAL;
    pn_check_report rep;
    std::memset(&rep, 0, sizeof(rep));
    rep.checked = k;
    rep.host_seconds = (double)b.done_ns.load() * 1e-9;
    if (rc == PN_OK) {
        auto dots = [](const double* v, int64_t stride, double* d) {
            // S1h.S2h, S1h.Lh, S2h.Lh with current norms; 0 where a norm is 0
            double s1[3], s2[3], l[3];
            for (int c = 0; c < 3; ++c) {
                s1[c] = v[(1 + c) * stride];
                s2[c] = v[(4 + c) * stride];
                l[c] = v[(7 + c) * stride];
            }
            const double n1 = std::sqrt(s1[0] * s1[0] + s1[1] * s1[1] + s1[2] * s1[2]);
            const double n2 = std::sqrt(s2[0] * s2[0] + s2[1] * s2[1] + s2[2] * s2[2]);
            const double nl = std::sqrt(l[0] * l[0] + l[1] * l[1] + l[2] * l[2]);
            const double a = s1[0] * s2[0] + s1[1] * s2[1] + s1[2] * s2[2];
            const double bb = s1[0] * l[0] + s1[1] * l[1] + s1[2] * l[2];
            const double cc = s2[0] * l[0] + s2[1] * l[1] + s2[2] * l[2];
            d[0] = (n1 > 0 && n2 > 0) ? a / (n1 * n2) : 0.0;
            d[1] = (n1 > 0 && nl > 0) ? bb / (n1 * nl) : 0.0;
            d[2] = (n2 > 0 && nl > 0) ? cc / (n2 * nl) : 0.0;
        };
        for (int64_t i = 0; i < k; ++i) {
            const Result& r = b.res[i];
            int flag = 0;
            if (status_gpu[i] != r.status) {
                ++rep.status_mismatches;
                flag |= 1;
            }
            if (steps_gpu[i] != r.acc || steps_gpu[ld_gpu + i] != r.rej) ++rep.step_mismatches;
            if (status_gpu[i] == PN_ST_OK && r.status == PN_ST_OK) {
                double dg[3], dc[3];
                dots(y_gpu + i, ld_gpu, dg);
                dots(r.y, 1, dc);
                double dd = 0.0;
                for (int c = 0; c < 3; ++c) {
                    const double e = std::fabs(dg[c] - dc[c]);
                    dd = (e > dd || e != e) ? e : dd;
                }
                if (!(dd <= dot_tol)) flag |= 2;
                if (dd > rep.max_dot_diff || dd != dd) rep.max_dot_diff = dd;
            }
            if (flag) ++rep.flagged;
            if (flags) flags[i] = flag;
        }
    }
    if (report) *report = rep;
    delete handle;
    return rc;
}

}  // extern "C"
