// pn_order.hip -- the order in which the persistent schedule hands inspirals
// to lanes: longest first, by a leading-order estimate of each inspiral's
// number of steps (pn_cost_order in include/pn.h).
//
// Lanes of one wave step together, so a wave runs as long as its longest
// inspiral; once no inspiral is left to hand out, the waves drain while the
// last ones finish.  Handing out the longest inspirals first puts short ones
// at the end, where the drain is.  The estimate:
//   an adaptive method of order p takes steps h with h^p |y^(p)| ~ tol, so it
//   needs about tol^(-1/p) times the integral of |y^(p)|^(1/p) dt steps.  A
//   spin precessing at the rate Omega_i with amplitude a_i (its component
//   normal to the precession axis) has |y^(5)| = a_i Omega_i^5, which gives
//   a_i^(1/5) Omega_i per unit time.  At leading order (the L_hat part of
//   Eq. (4) and the Newtonian chirp of Eq. (1), d omega/dt = (96/5) eta
//   M^(5/3) omega^(11/3)) the precession angle from omega0 to omega_f is
//   (5/192) (4 + 3 m_j/m_i) (1/omega0 - 1/omega_f) / M, independent of eta.
//   The key is the larger of the two spins' a_i^(1/5) times that angle, with
//   the total angular momentum J = eta M^(5/3) omega0^(-1/3) L_hat + S1 + S2
//   at the start as the precession axis.  Only the ranking matters, so
//   constant factors are dropped.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <rocprim/device/device_radix_sort.hpp>

#include "pn.h"

namespace pn_order {

constexpr int kBlock = 256;

// |v| sin(angle between v and the unit vector a)
__device__ __forceinline__ double normal_part(double v0, double v1, double v2, double a0, double a1, double a2) {
    const double vv = v0 * v0 + v1 * v1 + v2 * v2;
    const double va = v0 * a0 + v1 * a1 + v2 * a2;
    return __builtin_sqrt(__builtin_fmax(vv - va * va, 0.0));
}

__global__ void cost_key_kernel(int64_t n, int64_t ld, const double* __restrict__ m, const double* __restrict__ S,
                                const double* __restrict__ L, const double* __restrict__ w0, double omega_f,
                                uint16_t* __restrict__ key, int32_t* __restrict__ idx,
                                double* __restrict__ packed) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const double m1 = m[i], m2 = m[ld + i], w = w0[i];
    const double s10 = S[i], s11 = S[ld + i], s12 = S[2 * ld + i];
    const double s20 = S[3 * ld + i], s21 = S[4 * ld + i], s22 = S[5 * ld + i];
    const double l0 = L[i], l1 = L[ld + i], l2 = L[2 * ld + i];
    idx[i] = (int32_t)i;
    if (packed) {
        // the inputs as one 128-byte record: each lane's eight 16-byte stores
        // fill its own cache line, so the lines leave L2 whole
        double2* r = (double2*)(packed + i * 16);
        r[0] = make_double2(m1, m2);
        r[1] = make_double2(w, s10);
        r[2] = make_double2(s11, s12);
        r[3] = make_double2(s20, s21);
        r[4] = make_double2(s22, l0);
        r[5] = make_double2(l1, l2);
        r[6] = make_double2(0.0, 0.0);
        r[7] = make_double2(0.0, 0.0);
    }
    double k = 0.0;       // inputs the integrator refuses, or that finish at once: last
    if (m1 > 0.0 && m2 > 0.0 && w > 0.0 && (omega_f <= 0.0 || w < omega_f)) {
        const double M = m1 + m2;
        const double eta = m1 * m2 / (M * M);
        const double lmag = eta * pow(M, 5.0 / 3.0) * pow(w, -1.0 / 3.0);
        const double j0 = lmag * l0 + s10 + s20, j1 = lmag * l1 + s11 + s21, j2 = lmag * l2 + s12 + s22;
        const double jn = __builtin_sqrt(j0 * j0 + j1 * j1 + j2 * j2);
        const double span = (omega_f > 0.0 ? 1.0 / w - 1.0 / omega_f : 1.0 / w) / M;
        if (jn > 0.0 && __builtin_isfinite(jn) && __builtin_isfinite(span)) {
            const double a0 = j0 / jn, a1 = j1 / jn, a2 = j2 / jn;
            const double k1 = (4.0 + 3.0 * m2 / m1) * pow(normal_part(s10, s11, s12, a0, a1, a2), 0.2);
            const double k2 = (4.0 + 3.0 * m1 / m2) * pow(normal_part(s20, s21, s22, a0, a1, a2), 0.2);
            const double kk = span * __builtin_fmax(k1, k2);
            if (__builtin_isfinite(kk)) k = kk;
        }
    }
    // positive floats order as their bit patterns do; the upper 16 bits
    // (sign, exponent and 7 mantissa bits) rank the keys to within 1 %, far
    // finer than the estimate itself, and halve the sort's passes
    const float kf = (float)k;
    key[i] = kf > 0.0f ? (uint16_t)(__float_as_uint(kf) >> 16) : (uint16_t)0;
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

size_t sort_temp_bytes(int64_t n) {
    size_t bytes = 0;
    if (rocprim::radix_sort_pairs_desc(nullptr, bytes, (const uint16_t*)nullptr, (uint16_t*)nullptr,
                                       (const int32_t*)nullptr, (int32_t*)nullptr, (size_t)n, 0, 16) != hipSuccess)
        return 0;
    return bytes;
}

}  // namespace pn_order

using namespace pn_order;

extern "C" {

size_t pn_cost_order_workspace_bytes(int64_t n) {
    if (n < 0 || n > INT32_MAX) return 0;
    if (n == 0) return 0;
    const size_t t = sort_temp_bytes(n);
    if (t == 0) return 0;
    return 3 * align256((size_t)n * 4) + align256(t);
}

int pn_cost_order(int64_t n, int64_t ld, const double* m, const double* S0, const double* L0, const double* omega0,
                  double omega_f, int32_t* order, void* workspace, size_t ws_bytes, double* packed,
                  void* stream) {
    if (n < 0 || n > INT32_MAX || ld < n || ld > PN_MAX_N) return PN_EINVAL;
    if (!(omega_f == omega_f)) return PN_EINVAL;
    if (n == 0) return PN_OK;
    if (!m || !S0 || !L0 || !omega0 || !order || !workspace) return PN_EINVAL;
    if (((uintptr_t)packed & 15) != 0) return PN_EINVAL;
    const size_t need = pn_cost_order_workspace_bytes(n);
    if (need == 0 || ws_bytes < need) return PN_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    char* w = (char*)workspace;
    const size_t a = align256((size_t)n * 4);
    uint16_t* key_in = (uint16_t*)w;
    uint16_t* key_out = (uint16_t*)(w + a);
    int32_t* idx_in = (int32_t*)(w + 2 * a);
    void* tmp = (void*)(w + 3 * a);
    size_t tmp_bytes = need - 3 * a;
    const unsigned grid = (unsigned)((n + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(cost_key_kernel, dim3(grid), dim3(kBlock), 0, s, n, ld, m, S0, L0, omega0, omega_f, key_in,
                       idx_in, packed);
    if (hipGetLastError() != hipSuccess) return PN_EHIP;
    if (rocprim::radix_sort_pairs_desc(tmp, tmp_bytes, key_in, key_out, idx_in, order, (size_t)n, 0, 16, s) !=
        hipSuccess)
        return PN_EHIP;
    return hipGetLastError() == hipSuccess ? PN_OK : PN_EHIP;
}

}  // extern "C"
