// pn_generate.hip -- initial data drawn on the GPU from the counter-based
// Philox4x64-10 generator (Salmon, Moraes, Dror & Shaw, SC11): masses,
// isotropic spins (Marsaglia's method) and initial frequencies, one lane per
// inspiral, each inspiral from its own counter range.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>

#include "pn.h"

namespace pn {

int device_ready();   // pn_lib.hip: PN_OK when a gfx950 device is current

namespace {

constexpr int kBlock = 256;
constexpr int kMaxAttempts = 64;

constexpr uint64_t kM0 = 0xD2E7470EE14C6C93ull, kM1 = 0xCA5A826395121157ull;
constexpr uint64_t kW0 = 0x9E3779B97F4A7C15ull, kW1 = 0xBB67AE8584CAA73Bull;

struct U4 {
    uint64_t x[4];
};

// ten rounds of (x0, x1, x2, x3) -> (hi(M1 x2) ^ x1 ^ k0, lo(M1 x2),
// hi(M0 x0) ^ x3 ^ k1, lo(M0 x0)), the key advanced between rounds
__device__ __forceinline__ U4 philox(uint64_t c0, uint64_t c1, uint64_t k0, uint64_t k1) {
    uint64_t x0 = c0, x1 = c1, x2 = 0, x3 = 0;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) { k0 += kW0; k1 += kW1; }
        const uint64_t hi0 = __umul64hi(kM0, x0), lo0 = kM0 * x0;
        const uint64_t hi1 = __umul64hi(kM1, x2), lo1 = kM1 * x2;
        x0 = hi1 ^ x1 ^ k0;
        x1 = lo1;
        x2 = hi0 ^ x3 ^ k1;
        x3 = lo0;
    }
    return U4{{x0, x1, x2, x3}};
}

__device__ __forceinline__ double uniform(uint64_t w) { return (double)(w >> 11) * 0x1p-53; }

// products and sums rounded one by one, as the definition writes them
__device__ __forceinline__ double affine(double lo, double hi, double u) {
#pragma clang fp contract(off)
    return lo + (hi - lo) * u;
}

__device__ __forceinline__ void sphere(uint64_t i, uint64_t first_block, uint64_t k0, double* s) {
#pragma clang fp contract(off)
    s[0] = 0.0; s[1] = 0.0; s[2] = 1.0;
    for (int a = 0; a < kMaxAttempts; a += 2) {
        const U4 w = philox(i, first_block + (uint64_t)(a / 2), k0, 0);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const double u1 = 2.0 * uniform(w.x[2 * h]) - 1.0;
            const double u2 = 2.0 * uniform(w.x[2 * h + 1]) - 1.0;
            const double q = u1 * u1 + u2 * u2;
            if (q < 1.0) {
                const double r = 2.0 * sqrt(1.0 - q);
                s[0] = u1 * r;
                s[1] = u2 * r;
                s[2] = 1.0 - 2.0 * q;
                return;
            }
        }
    }
}

__global__ __launch_bounds__(kBlock) void generate_kernel(int64_t n, int64_t ld, int64_t first, pn_gen_spec sp,
                                                          double* __restrict__ m, double* __restrict__ S,
                                                          double* __restrict__ L, double* __restrict__ w0) {
#pragma clang fp contract(off)
    const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (j >= n) return;
    const uint64_t i = (uint64_t)(first + j);
    const uint64_t key = sp.seed;
    const U4 b = philox(i, 0, key, 0);
    const double q = affine(sp.q_lo, sp.q_hi, uniform(b.x[0]));
    const double c1 = affine(sp.chi1_lo, sp.chi1_hi, uniform(b.x[1]));
    const double c2 = affine(sp.chi2_lo, sp.chi2_hi, uniform(b.x[2]));
    const double om = affine(sp.omega0_lo, sp.omega0_hi, uniform(b.x[3]));
    const double m1 = q / (1.0 + q);
    const double m2 = 1.0 / (1.0 + q);
    double s1[3], s2[3];
    sphere(i, 1, key, s1);
    sphere(i, 1 + kMaxAttempts / 2, key, s2);
    const double a1 = c1 * (m1 * m1);
    const double a2 = c2 * (m2 * m2);
    m[j] = m1;
    m[ld + j] = m2;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        S[c * ld + j] = a1 * s1[c];
        S[(3 + c) * ld + j] = a2 * s2[c];
        L[c * ld + j] = c == 2 ? 1.0 : 0.0;
    }
    w0[j] = om;
}

bool bad_range(double lo, double hi) { return !(std::isfinite(lo) && std::isfinite(hi) && lo <= hi); }

}  // namespace
}  // namespace pn

using namespace pn;

extern "C" int pn_generate(int64_t n, int64_t ld, int64_t first, const pn_gen_spec* spec, double* m, double* S0,
                           double* L0, double* omega0, void* stream) {
    if (n < 0 || ld < n || ld > PN_MAX_N || first < 0 || first > INT64_MAX - n || !spec) return PN_EINVAL;
    const pn_gen_spec& s = *spec;
    if (bad_range(s.q_lo, s.q_hi) || !(s.q_lo > 0.0) || bad_range(s.chi1_lo, s.chi1_hi) ||
        bad_range(s.chi2_lo, s.chi2_hi) || s.chi1_lo < 0.0 || s.chi1_hi > 1.0 || s.chi2_lo < 0.0 ||
        s.chi2_hi > 1.0 || bad_range(s.omega0_lo, s.omega0_hi) || !(s.omega0_lo > 0.0))
        return PN_EINVAL;
    if (n > 0 && (!m || !S0 || !L0 || !omega0)) return PN_EINVAL;
    if (n == 0) return PN_OK;
    const int rc = device_ready();
    if (rc != PN_OK) return rc;
    hipLaunchKernelGGL(generate_kernel, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                       (hipStream_t)stream, n, ld, first, s, m, S0, L0, omega0);
    return hipGetLastError() == hipSuccess ? PN_OK : PN_EHIP;
}
