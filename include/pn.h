/*
 * pn.h -- C interface of the MI355X (gfx950) batched post-Newtonian
 * inspiral integrator.
 *
 * The library integrates many independent binary-black-hole inspirals, each
 * the ODE system of the paper (Herrmann et al., arXiv:0908.3889, Sec. II):
 *   state  y = (omega, S1[3], S2[3], L_hat[3])
 *   Eq. (1) d omega/dt (to 3.5PN, with 1.5PN spin-orbit and 2PN spin-spin),
 *   Eq. (2) dS_i/dt = Omega_i x S_i,  Eq. (3) dL_hat/dt,
 *   Eq. (4) Omega_1 (and Omega_2 by 1 <-> 2),
 * from omega0 to omega_f with the adaptive Dormand-Prince method at error
 * tolerance tol and initial step h = 10 (Sec. II).  One GPU lane integrates
 * one inspiral at a time; a persistent kernel hands new inspirals to lanes
 * as theirs finish.
 *
 * Conventions for every entry point:
 *  - Arrays are structure-of-arrays of float64 (int32 where stated): component
 *    c of inspiral i lives at p[c*ld + i], with leading dimension ld >= n;
 *    0 <= n <= ld <= PN_MAX_N.
 *  - Every array pointer is a DEVICE pointer on the current HIP device,
 *    allocated and owned by the caller; the library never frees it.  Inputs
 *    are read only; outputs are written for every i < n.
 *  - `stream` is a hipStream_t (NULL = the default stream).  Calls are
 *    asynchronous on that stream: they return once the work is enqueued.  The
 *    library never synchronises the device (pn_autotune excepted: it reads
 *    its timers), prints or aborts.
 *  - The return value is PN_OK (0) when the work was enqueued, or a negative
 *    PN_E* code: PN_EINVAL for bad arguments (nothing is launched),
 *    PN_ENODEV when no usable gfx950 device is current, PN_EHIP when a HIP
 *    call or launch failed (checked after every launch).  pn_strerror()
 *    names a code.
 *  - Outcomes per inspiral go to status[i] (PN_ST_*), never to the return code.
 *  - Safe to call from several host threads on different streams.  The
 *    library keeps a small per-device context, created on first use: the
 *    device's compute-unit count and 5120 call slots of 512 bytes, each a
 *    work counter and the launch arguments of one persistent launch (the
 *    only device memory the library allocates).  Direct calls take the
 *    first 1024 slots in turn; before a slot is reused, the new call's
 *    stream waits for an event recorded after the launch that last used it,
 *    so any number of launches may be queued on any streams.  A call made
 *    while its stream is being captured into a HIP graph takes one of the
 *    other 4096 slots for good (every replay of the graph uses it); when
 *    those are used up such a call returns PN_EBUSY and launches nothing
 *    (pn_shutdown frees them, and with them every graph captured before).
 *    Replays of one graph must not overlap one another.
 */
#ifndef PN_H
#define PN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Largest n (and leading dimension) any entry point accepts: 2^36 inspirals,
 * far beyond one GPU's memory; larger values give PN_EINVAL. */
#define PN_MAX_N ((int64_t)1 << 36)

/* ---- return codes ---------------------------------------------------- */
#define PN_OK        0
#define PN_EINVAL   -1   /* invalid argument */
#define PN_ENODEV   -2   /* no usable device */
#define PN_EHIP     -3   /* a HIP runtime call or kernel launch failed */
#define PN_ENOMEM   -4   /* the library could not allocate its device context */
#define PN_EBUSY    -5   /* no call slot left for a launch captured into a graph */

/* ---- per-inspiral status codes (status[i]) --------------------------- */
#define PN_ST_OK                    0  /* reached omega_f (or t_end) */
#define PN_ST_DONE_AT_START         1  /* omega0 >= omega_f: no step, y_final = y0, t = 0 */
#define PN_ST_MAX_STEPS            -1  /* accepted + rejected steps reached max_steps */
#define PN_ST_H_UNDERFLOW          -2  /* step size fell below 1e-14 of the independent variable */
#define PN_ST_NONFINITE            -3  /* NaN error estimate or non-finite candidate state */
#define PN_ST_BAD_INPUT            -4  /* m_i <= 0, omega0 <= 0 or a non-finite input */
#define PN_ST_OMEGADOT_NONPOSITIVE -5  /* d omega/dt <= 0 at the start of a step */
#define PN_ST_TAPE_FULL            -6  /* pn_integrate_record: more accepted steps than cap_steps */

/* ---- which terms of Eqs. (1)-(4) are on (bitmask) --------------------- */
#define PN_TERM_PN       1   /* non-spinning corrections of Eq. (1), (M w)^{2/3} ... (M w)^{7/3} */
#define PN_TERM_SO_WDOT  2   /* spin-orbit term of Eq. (1) */
#define PN_TERM_SS_WDOT  4   /* spin-spin term of Eq. (1) */
#define PN_TERM_RR       8   /* d omega/dt itself; off => omega is constant */
#define PN_TERM_SO_PREC 16   /* the L_hat part of Eq. (4) */
#define PN_TERM_SS_PREC 32   /* the S_j - 3 (S_j . L_hat) L_hat part of Eq. (4) */
#define PN_TERM_ALL     63

/* ---- arithmetic ---------------------------------------------------------- */
#define PN_PREC_FP64        0  /* everything in FP64 */
#define PN_PREC_FP32_SPLIT  1  /* stages, right-hand sides, increments and error
                                  estimate in FP32; state, t, h, error norm, step
                                  control and the omega >= omega_f test in FP64
                                  (the FP32 increment is added to the FP64 state);
                                  the paper ran its GPU in single precision with a
                                  few computations in double (Sec. III) */
#define PN_PREC_FP32_STATE  2  /* as PN_PREC_FP32_SPLIT, but the state too is FP32:
                                  omega as a float plus the summed rounding of its
                                  increments (compensated summation, about 48
                                  bits), S1, S2, L_hat as floats; the phase of
                                  pn_integrate_phase is summed the same way; t, h,
                                  the error norm, the step control and the
                                  omega >= omega_f test stay FP64 */

/* ---- scheduling -------------------------------------------------------- */
#define PN_SCHED_PERSISTENT 0  /* resident grid; lanes take new inspirals as theirs finish */
#define PN_SCHED_STATIC     1  /* one lane per inspiral, no refill */

/* Options.  A zero-initialised struct (or a NULL pointer) gives the paper's
 * settings: adaptive Dormand-Prince, h0 = 10, all terms, omega_f termination. */
typedef struct pn_opts {
    double  h0;            /* initial step in units of M; <= 0 -> 10 (Sec. II) */
    double  h_fixed;       /* > 0: fixed step h_fixed, no error control */
    double  t_end;         /* > 0: integrate to t = t_end instead of omega_f */
    int64_t max_steps;     /* per inspiral, accepted + rejected; <= 0 -> 10,000,000 */
    int32_t terms;         /* PN_TERM_* mask; <= 0 -> PN_TERM_ALL */
    int32_t theta_literal; /* 0: theta_hat multiplies eta once in the 3PN term (the
                              expansion the paper cites); 1: the extra factor eta
                              exactly as printed in Eq. (1) */
    int32_t schedule;      /* PN_SCHED_* */
    int32_t block;         /* threads per block: 64, 128, 256 or 512; 0 -> 256 */
    int32_t waves_per_simd;/* persistent grid: waves per SIMD (1..8); 0 -> the
                              occupancy the kernel is compiled for (2 FP64, 3 FP32-split) */
    int32_t refill_min;    /* persistent: a wave refills once this many of its lanes
                              are idle (1..64), or all are; 0 -> 4 (each refill pass
                              costs the whole wave, so refilling in small batches
                              beats refilling every lane at once) */
    int32_t precision;     /* PN_PREC_*; 0 -> FP64 */
    const int32_t* order;  /* NULL, or device int32 [n]: the inspiral indices in the
                              order in which the schedule hands them to lanes (a
                              permutation of 0 .. n-1, e.g. from pn_cost_order).
                              Every output is written at the inspiral's own index,
                              so the results do not depend on the order, only the
                              speed does.  Entries outside [0, n) are skipped (that
                              slot integrates nothing); an index missing from the
                              array leaves its outputs unwritten.  Requires
                              n <= 2^31 - 1. */
    const double* packed;  /* NULL, or device double [n][16], 16-byte aligned: each
                              inspiral's inputs as one 128-byte record (m1, m2,
                              omega0, S1, S2, L_hat, then four zeros), as
                              pn_cost_order writes them.  When set, the kernels
                              read the inputs from here (one cache line per
                              inspiral) instead of from m, S0, L0, omega0 (whose
                              pointers are still checked); the records must hold
                              the same inputs, and the results are then the
                              same, bit for bit.  PN_EINVAL if misaligned. */
} pn_opts;

/*
 * pn_integrate -- integrate n inspirals from omega0 to omega_f (Sec. II).
 *
 * Inputs (device, float64, SoA with leading dimension ld):
 *   m      [2][ld]  masses m1, m2 (> 0).  The equations are scale free; the
 *                   paper fixes M = m1 + m2 = 1 (Sec. II).
 *   S0     [6][ld]  initial spins S1 (x,y,z), S2 (x,y,z); S_i = chi_i m_i^2 S_hat_i.
 *   L0     [3][ld]  initial unit orbital angular momentum direction L_hat.
 *   omega0 [ld]     initial orbital frequency (> 0).
 *   omega_f         termination frequency (> 0; ignored when opt->t_end > 0).
 *   tol             error tolerance: absolute and relative tolerance of the
 *                   root-mean-square error norm over the 10 state components
 *                   (> 0 unless opt->h_fixed > 0).
 * Outputs (device):
 *   y_final [10][ld] final state (omega, S1, S2, L_hat); omega = omega_f exactly
 *                    on PN_ST_OK.  On a failure status: the last accepted state.
 *   t_final [ld]     elapsed time t (units of M).
 *   steps   [3][ld]  int32: accepted steps (time steps + final omega-steps),
 *                    rejected steps, right-hand-side evaluations.
 *   status  [ld]     int32 PN_ST_* code.
 *   dots    [3][ld]  optional (may be NULL): S1_hat.S2_hat, S1_hat.L_hat,
 *                    S2_hat.L_hat of the final state (0 where a norm is 0),
 *                    the observables of Sec. V.
 * n = 0 is valid and launches nothing.
 */
int pn_integrate(int64_t n, int64_t ld,
                 const double* m, const double* S0, const double* L0, const double* omega0,
                 double omega_f, double tol, const pn_opts* opt,
                 double* y_final, double* t_final, int32_t* steps, int32_t* status,
                 double* dots, void* stream);

/*
 * pn_cost_order -- an order in which to hand the inspirals to lanes (for
 * pn_opts.order): longest first, by a leading-order estimate of each
 * inspiral's number of steps.  Lanes of a wave step together, and once every
 * inspiral has been handed out the waves drain while the last ones finish;
 * with the longest handed out first the drain is made of short ones
 * (Sec. IV: throughput depends on how evenly the work is spread).  The
 * estimate: an adaptive 5th-order method needs about the integral of
 * |d^5 y/dt^5|^(1/5) dt steps; a spin precessing at rate Omega_i with
 * amplitude a_i contributes a_i^(1/5) Omega_i to the integrand, and the
 * leading-order precession angle (the L_hat part of Eq. (4) over the
 * Newtonian chirp of Eq. (1)) from omega0 to omega_f is proportional to
 * (4 + 3 m_j/m_i)(1/omega0 - 1/omega_f)/M.  The key is the larger of the two
 * spins' a_i^(1/5) times that angle, a_i being the component of S_i normal
 * to the initial total angular momentum.  Inspirals that end at once
 * (omega0 >= omega_f) or that the integrator refuses come last.  Equal keys
 * keep their index order.
 * Inputs as pn_integrate (device, SoA, leading dimension ld); omega_f <= 0
 * ranks by 1/omega0 alone.  order [n]: device int32 output, a permutation of
 * 0 .. n-1.  workspace: device scratch of at least
 * pn_cost_order_workspace_bytes(n) bytes, caller-owned.  packed: NULL, or a
 * device double [n][16] output (16-byte aligned, caller-owned) that receives
 * the inputs as the 128-byte records of pn_opts.packed, written by the same
 * pass that reads them for the keys: in the cost order, the lanes of a
 * refill read inspirals far apart in memory, and from the SoA arrays each of
 * their 12 input words costs a cache line of its own.  Requires
 * n <= 2^31 - 1; PN_EINVAL for bad sizes, NULL pointers, a small workspace or
 * a misaligned packed.  The ranking only changes the speed of pn_integrate,
 * never its results.
 */
size_t pn_cost_order_workspace_bytes(int64_t n);
int pn_cost_order(int64_t n, int64_t ld, const double* m, const double* S0, const double* L0,
                  const double* omega0, double omega_f, int32_t* order, void* workspace,
                  size_t ws_bytes, double* packed, void* stream);

/*
 * The check of GPU results against the CPU on a subset (Sec. III: kernel
 * failures on the GPU go unreported, so the paper integrated part of each
 * population on the CPU as well and compared).  A host integrator of the
 * same method (Eqs. (1)-(4), adaptive Dormand-Prince with the same error
 * norm, step control and final stretch in omega, plain FP64 with the C
 * library's cube root and log) runs on host threads while the GPU works;
 * its final states agree with the FP64 kernels' to rounding.
 *
 * pn_check_integrate_host -- the host integrator itself, synchronously:
 *   arguments, layout and outputs as pn_integrate but in HOST memory (no
 *   dots); pn_opts.precision, schedule, block, waves_per_simd, refill_min
 *   and order are ignored (it always integrates in FP64).  nthreads <= 0:
 *   one thread per core this process may run on.
 * pn_check_start -- copies k sampled inspirals (host SoA arrays with leading
 *   dimension ld: m [2][ld], S0 [6][ld], L0 [3][ld], omega0 [ld]) and starts
 *   integrating them on nthreads host threads (<= 0: one per core this
 *   process may run on); returns at once with *handle set.  PN_EINVAL for
 *   bad sizes, pointers or options; PN_ENOMEM if no thread could be started.
 * pn_check_finish -- waits for those threads and compares: GPU outputs of the
 *   same k inspirals in the same order (host copies: y [10][ld_gpu],
 *   steps [3][ld_gpu], status [ld_gpu]).  An inspiral is flagged when its
 *   status differs (flag bit 1) or when, both being PN_ST_OK, one of its unit
 *   dot products S1h.S2h, S1h.Lh, S2h.Lh differs by more than dot_tol (bit 2;
 *   1e-8 is the FP64 parity bar, FP32 modes need about 1e-3).  Differing step
 *   counts are counted, not flagged.  flags: optional int32 [k] output;
 *   report: optional.  Frees the handle (also on PN_EINVAL).
 */
typedef struct pn_check pn_check;
typedef struct pn_check_report {
    int64_t checked;            /* inspirals integrated on the host */
    int64_t status_mismatches;
    int64_t step_mismatches;    /* accepted or rejected step counts differ */
    int64_t flagged;            /* inspirals with a status or dot-product disagreement */
    double  max_dot_diff;       /* largest |GPU - host| over the dot products (both OK) */
    double  host_seconds;       /* wall time of the host integration */
} pn_check_report;
int pn_check_integrate_host(int64_t n, int64_t ld, const double* m, const double* S0, const double* L0,
                            const double* omega0, double omega_f, double tol, const pn_opts* opt,
                            double* y_final, double* t_final, int32_t* steps, int32_t* status,
                            int32_t nthreads);
int pn_check_start(pn_check** handle, int64_t k, int64_t ld, const double* m, const double* S0,
                   const double* L0, const double* omega0, double omega_f, double tol,
                   const pn_opts* opt, int32_t nthreads);
int pn_check_finish(pn_check* handle, const double* y_gpu, const int32_t* steps_gpu,
                    const int32_t* status_gpu, int64_t ld_gpu, double dot_tol, int32_t* flags,
                    pn_check_report* report);

/*
 * pn_integrate_noalloc -- pn_integrate for callers that cannot allocate
 * device memory: code being captured into a HIP graph, tight serving loops,
 * harnesses that forbid hipMalloc.  Same arguments, kernels, outputs and
 * errors as pn_integrate, bit for bit; the caller still owns every input and
 * output.  The call allocates nothing: no hipMalloc or hipFree, no event, no
 * library context.  The only device memory besides the caller's buffers is a
 * fixed 512-byte scratch array in the library (the persistent launch's work
 * counter and launch descriptor), one copy per device, held until the
 * process ends; its size does not depend on n, so every n that pn_integrate
 * accepts (0 <= n <= ld <= PN_MAX_N) fits, and larger n is PN_EINVAL.  The
 * counter is cleared by a kernel on `stream` at the start of each call.
 * Every pn_integrate_noalloc call on a device shares that array: calls on one
 * stream are ordered and safe, but calls that overlap on one device (several
 * streams or threads without ordering between them, or a captured graph
 * replayed while another such call runs) race and give wrong outputs.  The
 * first call on a device looks up the array's device address
 * (hipGetSymbolAddress); PN_EHIP if that fails.
 */
int pn_integrate_noalloc(int64_t n, int64_t ld,
                         const double* m, const double* S0, const double* L0, const double* omega0,
                         double omega_f, double tol, const pn_opts* opt,
                         double* y_final, double* t_final, int32_t* steps, int32_t* status,
                         double* dots, void* stream);

/*
 * pn_integrate_phase -- pn_integrate that also integrates the orbital phase
 * Phi(t) = integral of omega dt from Phi(0) = 0 (a quantity the paper does not
 * use; the phase of waveform-style outputs).  Each accepted step adds h times
 * the 5th-order weights applied to the stage values of omega (times
 * dt/d omega on the final stretch in omega); Phi is left out of the error
 * norm, so the steps and every other output are bit-identical to
 * pn_integrate's.  phase [ld]: device float64 output, Phi at t_final (0 for
 * DONE_AT_START and BAD_INPUT; at the last accepted state for a failure).
 * In PN_PREC_FP32_SPLIT the per-step increment is formed in FP32 and summed
 * in FP64, like the state.  Other arguments, errors and layout as
 * pn_integrate; phase must not be NULL when n > 0.
 */
int pn_integrate_phase(int64_t n, int64_t ld,
                       const double* m, const double* S0, const double* L0, const double* omega0,
                       double omega_f, double tol, const pn_opts* opt,
                       double* y_final, double* t_final, int32_t* steps, int32_t* status,
                       double* dots, double* phase, void* stream);

/*
 * pn_autotune -- choose the launch shape of pn_integrate for a population:
 * times pn_integrate on its first `sample` inspirals (all n when sample <= 0
 * or sample > n) for every candidate refill threshold {2, 3, 4, 6} and block
 * size {128, 256} (waves per SIMD as compiled), `reps` times each (<= 0 ->
 * 2) after one warm-up run, and writes the fastest to *best: a copy of *opt
 * (or of the defaults when opt is NULL) with `block` and `refill_min` set.
 * The outcome of an integration does not depend on the launch shape, so the
 * choice only affects speed.  y_final .. dots: device outputs for the sample
 * (caller-owned, leading dimension ld, at least the sample's entries); they
 * hold an integration of the sample afterwards.  times_ms: optional host
 * array of 8 doubles, each candidate's mean time in the order (refill, block)
 * = (2,128), (2,256), (3,128), ... (6,256).  Unlike the other entry points
 * this call blocks: it synchronises `stream` to read its timers.
 */
int pn_autotune(int64_t n, int64_t ld, const double* m, const double* S0, const double* L0,
                const double* omega0, double omega_f, double tol, const pn_opts* opt, int64_t sample,
                int32_t reps, double* y_final, double* t_final, int32_t* steps, int32_t* status,
                double* dots, pn_opts* best, double* times_ms, void* stream);

/*
 * pn_shutdown -- frees the library's context on the current device (its
 * call slots and their events); the next call on that device creates it
 * again.  Call it only when no work of the library is queued or running on
 * the device, and not concurrently with other calls for that device; graphs
 * captured before it must not be replayed after it.  PN_OK also when there
 * is no context; PN_EHIP if freeing failed.
 */
int pn_shutdown(void);

/*
 * pn_fma_rate -- the device's sustained vector multiply-add rate, the
 * measured counterpart of the datasheet peaks that roofline fractions are
 * quoted against: eight independent FMA chains per lane, 16 x iters steps
 * each, on CUs x waves_per_simd blocks of 256 threads (waves_per_simd
 * 1..8, iters 1..2^20), in FP32 without packed instructions and in FP64.
 * Writes TFLOP/s (an FMA counted as 2) to *fp32_tflops and *fp64_tflops
 * (host pointers).  Allocates and frees a small device buffer and blocks
 * until its timers are read.
 */
int pn_fma_rate(int32_t waves_per_simd, int32_t iters, double* fp32_tflops, double* fp64_tflops, void* stream);

/*
 * pn_fma_lanes -- the FP64 chains of pn_fma_rate on the first active_lanes
 * (0..64) lanes of every wave only, one wave per SIMD (one block of 256 per
 * CU), once: a launch whose lane FLOPs are known, for calibrating instruction
 * and FLOP counters on partly active waves (a profiler reads the counters;
 * the library only launches).  Writes the lane FLOPs of the launch (an FMA
 * counted as 2) to *lane_flop and its duration to *ms (host pointers).
 * Allocates and frees a small device buffer and blocks until the timer is
 * read.
 */
int pn_fma_lanes(int32_t active_lanes, int32_t iters, double* lane_flop, double* ms, void* stream);

/*
 * pn_rhs -- Eqs. (1)-(4) evaluated pointwise, dy/dt at y, for testing the
 * right-hand side on its own.  m [2][ld], y [10][ld] -> dydt [10][ld].
 * `terms`/`theta_literal` as in pn_opts (opt may be NULL).
 */
int pn_rhs(int64_t n, int64_t ld, const double* m, const double* y, double* dydt,
           const pn_opts* opt, void* stream);

/*
 * pn_observables -- unit-vector scalar products of Sec. V:
 * y [10][ld] -> dots [3][ld] = (S1_hat.S2_hat, S1_hat.L_hat, S2_hat.L_hat),
 * each 0 where one of the norms is 0.
 */
int pn_observables(int64_t n, int64_t ld, const double* y, double* dots, void* stream);

/*
 * The discrete adjoint.
 *
 * pn_integrate_record -- pn_integrate (FP64, omega_f termination) that also
 * writes, per inspiral i, a tape of pn_tape_stride(cap_steps, ckpt_every)
 * doubles at tape + i * stride: [n_t, n_w, h_0 .. h_{cap-1}, y(0), y(K),
 * y(2K), ...] -- the number of accepted time steps and omega-steps, every
 * accepted step size, and the state every K = ckpt_every accepted steps.
 * An inspiral with more than cap_steps accepted steps ends with status
 * PN_ST_TAPE_FULL.  tape is a device buffer of n * stride doubles (caller
 * owned).  Other arguments as pn_integrate; opt->precision must be FP64 and
 * opt->t_end 0.
 */
size_t pn_tape_stride(int64_t cap_steps, int32_t ckpt_every);
int pn_integrate_record(int64_t n, int64_t ld,
                        const double* m, const double* S0, const double* L0, const double* omega0,
                        double omega_f, double tol, const pn_opts* opt,
                        double* y_final, double* t_final, int32_t* steps, int32_t* status,
                        double* dots, double* tape, int64_t cap_steps, int32_t ckpt_every,
                        void* stream);

/*
 * pn_integrate_adjoint -- reverse-mode derivative of the recorded integration
 * with the accepted step sizes held fixed (the discrete adjoint of the
 * Dormand-Prince map that produced y_final, t_final).  For the loss
 *   L = sum_i gy_final[:, i] . y_final[:, i] + gt_final[i] t_final[i]
 * it writes dL/dm [2][ld], dL/dS0 [6][ld], dL/dL0 [3][ld], dL/domega0 [ld].
 * The last omega-step ends on omega_f, so its size depends on the state and
 * the final omega carries no derivative.
 *   m, tape, cap_steps, ckpt_every, status: the inputs and outputs of the
 *     pn_integrate_record call (same masses, same opt->terms/theta_literal);
 *   gy_final [10][ld], gt_final [ld] (may be NULL = 0);
 *   workspace: device buffer of at least pn_adjoint_workspace_bytes(n, K)
 *     bytes (the replayed states of one checkpoint segment per inspiral);
 *   order: optional device permutation of [0, n) giving the order in which
 *     inspirals are assigned to lanes (e.g. sorted by step count, so that a
 *     wave's lanes run segments of equal length); NULL = identity.  Entries
 *     outside [0, n) are skipped, so an inspiral that a non-permutation
 *     misses gets no output.
 * Inspirals with status DONE_AT_START get the identity (dL/dS0 = gy, ...,
 * dL/dm = 0); any other non-OK status gets NaN, and so does an OK inspiral
 * whose tape row does not hold the counts of a recorded run (non-integer or
 * negative, or more than cap_steps steps): the tape is never read beyond
 * its row.
 */
size_t pn_adjoint_workspace_bytes(int64_t n, int32_t ckpt_every);
int pn_integrate_adjoint(int64_t n, int64_t ld, const double* m, double omega_f, const pn_opts* opt,
                         const double* tape, int64_t cap_steps, int32_t ckpt_every,
                         const int32_t* status, const double* gy_final, const double* gt_final,
                         double* g_m, double* g_S0, double* g_L0, double* g_omega0,
                         double* workspace, size_t ws_bytes, const int32_t* order, void* stream);

/*
 * pn_ckpt_bytes -- bytes of the tape of n inspirals recorded with cap_steps
 * and ckpt_every (n * pn_tape_stride(cap_steps, ckpt_every) doubles); 0 for
 * sizes the record call refuses.
 */
size_t pn_ckpt_bytes(int64_t n, int64_t cap_steps, int32_t ckpt_every);

/*
 * pn_integrate_replay -- the recorded integration's map with its step sizes
 * frozen, evaluated at any initial state: from (m, S0, L0, omega0) it takes
 * the n_t time steps h_0 .. h_{n_t-1} of the tape, then its n_w omega-steps,
 * the last of size omega_f - omega, and ends on omega_f (the Dormand-Prince
 * steps of Sec. II without error control; the map that pn_integrate_adjoint
 * differentiates).  Central differences of this map check the adjoint with
 * the steps held fixed.  tape, cap_steps, ckpt_every: as recorded by
 * pn_integrate_record (only the counts and step sizes are read).  status:
 * the recorded run's statuses, or NULL when every inspiral ended PN_ST_OK;
 * DONE_AT_START keeps the initial state (t = 0), any other failure gives NaN.
 * Outputs y_final [10][ld], t_final [ld] (device).  A row that does not hold
 * the counts of a recorded run, or inputs that pn_integrate refuses, give
 * NaN outputs.  opt: terms and theta_literal as recorded; precision FP64, no
 * t_end, no h_fixed (else PN_EINVAL).
 */
int pn_integrate_replay(int64_t n, int64_t ld, const double* m, const double* S0, const double* L0,
                        const double* omega0, double omega_f, const pn_opts* opt, const double* tape,
                        int64_t cap_steps, int32_t ckpt_every, const int32_t* status, double* y_final,
                        double* t_final,
                        void* stream);

/*
 * The statistics of Sec. V over per-inspiral values, e.g. the dot products
 * that pn_integrate writes to `dots` (final) and pn_observables gives for the
 * initial state.  All arrays are device float64 SoA with leading dimension
 * ld >= n; component c of entry i at x[c*ld + i], c < ncomp (1..16).  Every
 * result is written to caller-owned device memory; results are deterministic
 * (fixed reduction trees, independent of the device's CU count).  Return
 * codes as for pn_integrate.  n = 0 writes zero counts and NaN for every
 * floating result.
 *
 * pn_histogram -- counts[c][b] = number of entries with e_b <= x < e_{b+1},
 * e_b = lo + b*(hi - lo)/nbins (computed as a product then a sum, e_nbins =
 * hi, the last bin closed); entries outside [lo, hi] or NaN are not counted
 * (Sec. V: 20 and 100 bins on [-1, 1]).  counts: int64 [ncomp][nbins],
 * nbins 1..4096, lo < hi finite.
 */
int pn_histogram(int64_t n, int64_t ld, const double* x, int32_t ncomp, int32_t nbins, double lo, double hi,
                 int64_t* counts, void* stream);

/*
 * pn_histogram2d -- the bivariate histogram of (x[c], y[c]) with the bins of
 * pn_histogram in both dimensions (Sec. V: initial against final value, 79
 * bins): counts int64 [ncomp][nbins (x)][nbins (y)], nbins 1..128; an entry
 * counts only if both values are in [lo, hi].
 */
int pn_histogram2d(int64_t n, int64_t ld, const double* x, const double* y, int32_t ncomp, int32_t nbins,
                   double lo, double hi, int64_t* counts, void* stream);

/*
 * pn_pearson -- for each component pair (x[c], y[c]): out[c][0..4] = mean x,
 * mean y, standard deviation of x and of y (with 1/(n-1)), and the Pearson
 * product-moment coefficient r (Sec. V), from two passes (means, then
 * centred sums).  workspace: device buffer of pn_stats_workspace_bytes(n,
 * ncomp, 0) bytes.  n = 1 gives NaN deviations and r.
 */
int pn_pearson(int64_t n, int64_t ld, const double* x, const double* y, int32_t ncomp, double* out,
               void* workspace, size_t ws_bytes, void* stream);

/*
 * pn_kde -- the Gaussian kernel density estimator of Sec. V on ngrid points
 * g_k = lo + k*(hi - lo)/(ngrid - 1):
 *   out[c][k] = 1/(n h_c) sum_j exp(-(g_k - x[c][j])^2 / (2 h_c^2)) / sqrt(2 pi),
 * with Silverman's bandwidth h_c = 1.06 sigma_c n^(-1/5); sigma_c is read
 * from the device at sigma[c * sigma_stride] (e.g. the standard deviations
 * that pn_pearson wrote: sigma = out + 2, stride 5).  ngrid 2..4096.
 * workspace: pn_stats_workspace_bytes(n, ncomp, ngrid) bytes.
 */
int pn_kde(int64_t n, int64_t ld, const double* x, int32_t ncomp, const double* sigma, int64_t sigma_stride,
           int32_t ngrid, double lo, double hi, double* out, void* workspace, size_t ws_bytes, void* stream);

/*
 * pn_ks_uniform -- the Kolmogorov-Smirnov test of each component against the
 * uniform distribution on [lo, hi] (Sec. V): out[c][0] = D = max_i max(i/n -
 * F(x_(i)), F(x_(i)) - (i-1)/n) over the sorted values, F(x) = (x - lo)/(hi - lo);
 * out[c][1] = the asymptotic p-value P(K > sqrt(n) D) of the Kolmogorov
 * distribution.  The values must not be NaN.  workspace:
 * pn_ks_workspace_bytes(n) bytes (a sorted copy and the sort's scratch).
 */
size_t pn_ks_workspace_bytes(int64_t n);
int pn_ks_uniform(int64_t n, int64_t ld, const double* x, int32_t ncomp, double lo, double hi, double* out,
                  void* workspace, size_t ws_bytes, void* stream);

/* Workspace bytes of pn_pearson (ngrid = 0) and pn_kde (ngrid > 0). */
size_t pn_stats_workspace_bytes(int64_t n, int32_t ncomp, int32_t ngrid);

/*
 * On-device initial data (Sec. II, V): the population that pn_integrate takes,
 * drawn on the GPU from the counter-based Philox4x64-10 generator (Salmon et
 * al., SC11) with key (seed, 0).  Inspiral i (global index first + i) draws
 * only from the blocks at counters (first + i, k, 0, 0): block 0 gives the
 * uniforms u of q, chi_1, chi_2, omega0; blocks 1..32 the Marsaglia (1972)
 * attempts for S_hat_1 (two per block), blocks 33..64 those for S_hat_2; a
 * uniform is (x >> 11) 2^-53; after 64 rejected attempts S_hat = (0, 0, 1).
 * Each parameter is lo + (hi - lo) u (fixed when lo == hi).  Then M = 1,
 * m1 = q/(1 + q), m2 = 1/(1 + q), S_i = chi_i m_i^2 S_hat_i, L_hat = z.
 * The same (seed, index) always gives the same inspiral, bit for bit,
 * whatever n, first or the launch shape.
 */
typedef struct pn_gen_spec {
    double   q_lo, q_hi;            /* mass ratio m1/m2 */
    double   chi1_lo, chi1_hi;      /* Kerr parameters in [0, 1] */
    double   chi2_lo, chi2_hi;
    double   omega0_lo, omega0_hi;  /* initial orbital frequency (> 0) */
    uint64_t seed;
} pn_gen_spec;

/* pn_generate -- write m [2][ld], S0 [6][ld], L0 [3][ld], omega0 [ld]
 * (device, caller-owned) for inspirals first .. first + n - 1.
 * PN_EINVAL for q_lo <= 0, chi outside [0, 1], omega0_lo <= 0, lo > hi or
 * non-finite bounds. */
int pn_generate(int64_t n, int64_t ld, int64_t first, const pn_gen_spec* spec, double* m, double* S0,
                double* L0, double* omega0, void* stream);

/* Name of a PN_* return code (static string). */
const char* pn_strerror(int code);

/* Library version string (static). */
const char* pn_version(void);

#ifdef __cplusplus
}
#endif

#endif /* PN_H */
