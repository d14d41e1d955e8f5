// pn_stats.hip -- the statistics of Sec. V over per-inspiral values on the
// GPU: equal-width and bivariate histograms, the Pearson coefficient, the
// Gaussian kernel density estimator with Silverman's bandwidth, and the
// Kolmogorov-Smirnov statistic against the uniform law.
//
// Every reduction runs over a fixed grid of kPart partial results combined
// in a fixed order, so results do not depend on the device's size or on
// scheduling.  Histogram counts use integer atomics (order-free).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>

#include <rocprim/device/device_radix_sort.hpp>

#include "pn.h"

namespace pn {

int device_ready();   // pn_lib.hip: PN_OK when a gfx950 device is current

namespace {

constexpr int kBlock = 256;
constexpr int kPart = 512;          // partial results per component
constexpr int kMaxComp = 16;

// ---------------------------------------------------------------------------
// histograms
// ---------------------------------------------------------------------------

// lo + k*step as a rounded product and then a rounded sum (contraction into
// a fused multiply-add is switched off here)
__device__ __forceinline__ double affine(double k, double step, double lo) {
#pragma clang fp contract(off)
    return k * step + lo;
}

// bin edge e_b = lo + b*step, e_nbins = hi
__device__ __forceinline__ double edge(int b, int nbins, double lo, double hi, double step) {
    return b == nbins ? hi : affine((double)b, step, lo);
}

// the bin of lo <= v <= hi: an estimate from the quotient, corrected against
// the edges themselves
__device__ __forceinline__ int bin_of(double v, int nbins, double lo, double hi, double step) {
    int b = (int)((v - lo) / step);
    b = b < 0 ? 0 : (b > nbins - 1 ? nbins - 1 : b);
    while (b > 0 && v < edge(b, nbins, lo, hi, step)) --b;
    while (b < nbins - 1 && v >= edge(b + 1, nbins, lo, hi, step)) ++b;
    return b;
}

__global__ void zero_i64(int64_t* p, int64_t count) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

__global__ __launch_bounds__(kBlock) void hist_kernel(int64_t n, int64_t ld, const double* __restrict__ x, int nbins,
                                                      double lo, double hi, double step, int64_t* __restrict__ counts) {
    extern __shared__ unsigned int sh[];
    const int c = blockIdx.y;
    for (int b = threadIdx.x; b < nbins; b += kBlock) sh[b] = 0u;
    __syncthreads();
    const double* xc = x + (int64_t)c * ld;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
        const double v = xc[i];
        if (v >= lo && v <= hi) atomicAdd(&sh[bin_of(v, nbins, lo, hi, step)], 1u);
    }
    __syncthreads();
    for (int b = threadIdx.x; b < nbins; b += kBlock)
        if (sh[b]) atomicAdd((unsigned long long*)&counts[(int64_t)c * nbins + b], (unsigned long long)sh[b]);
}

__global__ __launch_bounds__(kBlock) void hist2d_kernel(int64_t n, int64_t ld, const double* __restrict__ x,
                                                        const double* __restrict__ y, int nbins, double lo, double hi,
                                                        double step, int64_t* __restrict__ counts) {
    extern __shared__ unsigned int sh[];
    const int c = blockIdx.y;
    const int nb2 = nbins * nbins;
    for (int b = threadIdx.x; b < nb2; b += kBlock) sh[b] = 0u;
    __syncthreads();
    const double* xc = x + (int64_t)c * ld;
    const double* yc = y + (int64_t)c * ld;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
        const double u = xc[i], v = yc[i];
        if (u >= lo && u <= hi && v >= lo && v <= hi)
            atomicAdd(&sh[bin_of(u, nbins, lo, hi, step) * nbins + bin_of(v, nbins, lo, hi, step)], 1u);
    }
    __syncthreads();
    for (int b = threadIdx.x; b < nb2; b += kBlock)
        if (sh[b]) atomicAdd((unsigned long long*)&counts[(int64_t)c * nb2 + b], (unsigned long long)sh[b]);
}

// ---------------------------------------------------------------------------
// fixed-order block reductions
// ---------------------------------------------------------------------------

template <int K>
__device__ __forceinline__ void block_sum(double (&v)[K], double (*sh)[kBlock]) {
#pragma unroll
    for (int k = 0; k < K; ++k) sh[k][threadIdx.x] = v[k];
    __syncthreads();
    for (int s = kBlock / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
#pragma unroll
            for (int k = 0; k < K; ++k) sh[k][threadIdx.x] += sh[k][threadIdx.x + s];
        }
        __syncthreads();
    }
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = sh[k][0];
    __syncthreads();
}

__device__ __forceinline__ double block_max(double v, double* sh) {
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int s = kBlock / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] = __builtin_fmax(sh[threadIdx.x], sh[threadIdx.x + s]);
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

// ---------------------------------------------------------------------------
// Pearson: pass 1 sums, pass 2 centred sums (workspace: part[c][kPart][3],
// then mean[c][2])
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(kBlock) void sums_kernel(int64_t n, int64_t ld, const double* __restrict__ x,
                                                      const double* __restrict__ y, double* __restrict__ part) {
    __shared__ double sh[2][kBlock];
    const int c = blockIdx.y;
    const double* xc = x + (int64_t)c * ld;
    const double* yc = y + (int64_t)c * ld;
    double v[2] = {0.0, 0.0};
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)kPart * kBlock) {
        v[0] += xc[i];
        v[1] += yc[i];
    }
    block_sum<2>(v, sh);
    if (threadIdx.x == 0) {
        part[((int64_t)c * kPart + blockIdx.x) * 3 + 0] = v[0];
        part[((int64_t)c * kPart + blockIdx.x) * 3 + 1] = v[1];
    }
}

__global__ __launch_bounds__(kBlock) void means_kernel(int64_t n, const double* __restrict__ part,
                                                       double* __restrict__ mean) {
    __shared__ double sh[2][kBlock];
    const int c = blockIdx.x;
    double v[2] = {0.0, 0.0};
    for (int b = threadIdx.x; b < kPart; b += kBlock) {
        v[0] += part[((int64_t)c * kPart + b) * 3 + 0];
        v[1] += part[((int64_t)c * kPart + b) * 3 + 1];
    }
    block_sum<2>(v, sh);
    if (threadIdx.x == 0) {
        mean[c * 2 + 0] = v[0] / (double)n;
        mean[c * 2 + 1] = v[1] / (double)n;
    }
}

__global__ __launch_bounds__(kBlock) void centred_kernel(int64_t n, int64_t ld, const double* __restrict__ x,
                                                         const double* __restrict__ y, const double* __restrict__ mean,
                                                         double* __restrict__ part) {
    __shared__ double sh[3][kBlock];
    const int c = blockIdx.y;
    const double* xc = x + (int64_t)c * ld;
    const double* yc = y + (int64_t)c * ld;
    const double mx = mean[c * 2], my = mean[c * 2 + 1];
    double v[3] = {0.0, 0.0, 0.0};
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)kPart * kBlock) {
        const double dx = xc[i] - mx, dy = yc[i] - my;
        v[0] += dx * dx;
        v[1] += dy * dy;
        v[2] += dx * dy;
    }
    block_sum<3>(v, sh);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < 3; ++k) part[((int64_t)c * kPart + blockIdx.x) * 3 + k] = v[k];
    }
}

__global__ __launch_bounds__(kBlock) void pearson_final_kernel(int64_t n, const double* __restrict__ part,
                                                               const double* __restrict__ mean, double* __restrict__ out) {
    __shared__ double sh[3][kBlock];
    const int c = blockIdx.x;
    double v[3] = {0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < kPart; b += kBlock) {
#pragma unroll
        for (int k = 0; k < 3; ++k) v[k] += part[((int64_t)c * kPart + b) * 3 + k];
    }
    block_sum<3>(v, sh);
    if (threadIdx.x == 0) {
        const double nm1 = (double)(n - 1);
        out[c * 5 + 0] = mean[c * 2];
        out[c * 5 + 1] = mean[c * 2 + 1];
        out[c * 5 + 2] = sqrt(v[0] / nm1);
        out[c * 5 + 3] = sqrt(v[1] / nm1);
        out[c * 5 + 4] = v[2] / sqrt(v[0] * v[1]);
    }
}

// ---------------------------------------------------------------------------
// KDE: block (b, c) takes a contiguous slice of the points and every grid
// point; partial sums part[c][b][g], combined in block order
// ---------------------------------------------------------------------------

__device__ __forceinline__ double kde_h(const double* sigma, int64_t stride, int c, double nfac) {
    return (1.06 * sigma[(int64_t)c * stride]) * nfac;
}

__global__ __launch_bounds__(kBlock) void kde_kernel(int64_t n, int64_t ld, const double* __restrict__ x,
                                                     const double* __restrict__ sigma, int64_t sstride, double nfac,
                                                     int ngrid, double lo, double gstep, double* __restrict__ part) {
    __shared__ double tile[kBlock];
    const int c = blockIdx.y;
    const double* xc = x + (int64_t)c * ld;
    const double ih = 1.0 / kde_h(sigma, sstride, c, nfac);
    const int64_t per = (n + kPart - 1) / kPart;
    const int64_t j0 = (int64_t)blockIdx.x * per;
    const int64_t j1 = (j0 + per < n) ? j0 + per : n;
    // one grid point per thread and pass; the block's slice of points is
    // staged through LDS once per pass
    for (int g0 = 0; g0 < ngrid; g0 += kBlock) {
        const int g = g0 + threadIdx.x;
        const double xg = affine((double)g, gstep, lo);
        double acc = 0.0;
        for (int64_t t0 = j0; t0 < j1; t0 += kBlock) {
            const int64_t j = t0 + threadIdx.x;
            tile[threadIdx.x] = j < j1 ? xc[j] : 0.0;
            __syncthreads();
            const int cnt = (int)((j1 - t0) < kBlock ? (j1 - t0) : kBlock);
            for (int k = 0; k < cnt; ++k) {
                const double u = (xg - tile[k]) * ih;
                acc += exp(-0.5 * u * u);
            }
            __syncthreads();
        }
        if (g < ngrid) part[((int64_t)c * kPart + blockIdx.x) * ngrid + g] = acc;
    }
}

__global__ __launch_bounds__(kBlock) void kde_final_kernel(int64_t n, const double* __restrict__ sigma, int64_t sstride,
                                                           double nfac, double sqrt2pi, int ngrid,
                                                           const double* __restrict__ part, double* __restrict__ out) {
    const int c = blockIdx.y;
    const int g = blockIdx.x * kBlock + threadIdx.x;
    if (g >= ngrid) return;
    const double h = kde_h(sigma, sstride, c, nfac);
    double s = 0.0;
    for (int b = 0; b < kPart; ++b) s += part[((int64_t)c * kPart + b) * ngrid + g];
    const double norm = 1.0 / (((double)n * h) * sqrt2pi);
    out[(int64_t)c * ngrid + g] = s * norm;
}

// ---------------------------------------------------------------------------
// Kolmogorov-Smirnov against U[lo, hi] on a sorted copy
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(kBlock) void ks_kernel(int64_t n, const double* __restrict__ xs, double lo, double hi,
                                                    double* __restrict__ part) {
    __shared__ double sh[kBlock];
    const double w = hi - lo;
    const double dn = (double)n;
    double d = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)kPart * kBlock) {
        const double F = (xs[i] - lo) / w;
        const double up = (double)(i + 1) / dn - F;
        const double dw = F - (double)i / dn;
        d = __builtin_fmax(d, __builtin_fmax(up, dw));
    }
    d = block_max(d, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = d;
}

// P(K > lam): alternating series for lam >= 1, theta-function form below
__device__ double kolmogorov_sf(double lam) {
    if (!(lam > 0.0)) return 1.0;
    const double pi = 3.14159265358979323846;
    double s = 0.0;
    if (lam >= 1.0) {
        for (int k = 1; k <= 100; ++k)
            s += ((k & 1) ? 2.0 : -2.0) * exp(-2.0 * (double)k * (double)k * lam * lam);
        return s < 0.0 ? 0.0 : (s > 1.0 ? 1.0 : s);
    }
    for (int k = 1; k <= 100; ++k) {
        const double m = (double)(2 * k - 1);
        s += exp(-(m * m) * (pi * pi) / (8.0 * lam * lam));
    }
    const double p = 1.0 - sqrt(2.0 * pi) / lam * s;
    return p < 0.0 ? 0.0 : (p > 1.0 ? 1.0 : p);
}

__global__ void ks_final_kernel(int64_t n, const double* __restrict__ part, double* __restrict__ out) {
    if (threadIdx.x != 0) return;
    double d = 0.0;
    for (int b = 0; b < kPart; ++b) d = __builtin_fmax(d, part[b]);
    out[0] = n > 0 ? d : __builtin_nan("");
    out[1] = n > 0 ? kolmogorov_sf(sqrt((double)n) * d) : __builtin_nan("");
}

__global__ void fill_nan(double* p, int count) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = __builtin_nan("");
}

int launched() { return hipGetLastError() == hipSuccess ? PN_OK : PN_EHIP; }

bool bad_common(int64_t n, int64_t ld, int32_t ncomp) {
    return n < 0 || ld < n || ld > PN_MAX_N || ncomp < 1 || ncomp > kMaxComp;
}

unsigned blocks_for(int64_t n) {
    const int64_t b = (n + kBlock - 1) / kBlock;
    return (unsigned)(b < 1 ? 1 : (b > 1024 ? 1024 : b));
}

size_t radix_temp_bytes(int64_t n) {
    size_t bytes = 0;
    if (n <= 0) return 0;
    if (rocprim::radix_sort_keys(nullptr, bytes, (const double*)nullptr, (double*)nullptr, (size_t)n) != hipSuccess)
        return 0;
    return bytes;
}

}  // namespace
}  // namespace pn

using namespace pn;

extern "C" {

int pn_histogram(int64_t n, int64_t ld, const double* x, int32_t ncomp, int32_t nbins, double lo, double hi,
                 int64_t* counts, void* stream) {
    if (bad_common(n, ld, ncomp) || nbins < 1 || nbins > 4096 || !(lo < hi) || !std::isfinite(lo) ||
        !std::isfinite(hi) || !counts || (n > 0 && !x))
        return PN_EINVAL;
    const int rc = device_ready();
    if (rc != PN_OK) return rc;
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(zero_i64, dim3(64), dim3(kBlock), 0, s, counts, (int64_t)ncomp * nbins);
    if (n > 0) {
        const double step = (hi - lo) / nbins;
        hipLaunchKernelGGL(hist_kernel, dim3(blocks_for(n), ncomp), dim3(kBlock), nbins * sizeof(unsigned), s, n, ld, x,
                           (int)nbins, lo, hi, step, counts);
    }
    return launched();
}

int pn_histogram2d(int64_t n, int64_t ld, const double* x, const double* y, int32_t ncomp, int32_t nbins,
                   double lo, double hi, int64_t* counts, void* stream) {
    if (bad_common(n, ld, ncomp) || nbins < 1 || nbins > 128 || !(lo < hi) || !std::isfinite(lo) ||
        !std::isfinite(hi) || !counts || (n > 0 && (!x || !y)))
        return PN_EINVAL;
    const int rc = device_ready();
    if (rc != PN_OK) return rc;
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(zero_i64, dim3(64), dim3(kBlock), 0, s, counts, (int64_t)ncomp * nbins * nbins);
    if (n > 0) {
        const double step = (hi - lo) / nbins;
        hipLaunchKernelGGL(hist2d_kernel, dim3(blocks_for(n), ncomp), dim3(kBlock),
                           (size_t)nbins * nbins * sizeof(unsigned), s, n, ld, x, y, (int)nbins, lo, hi, step, counts);
    }
    return launched();
}

size_t pn_stats_workspace_bytes(int64_t n, int32_t ncomp, int32_t ngrid) {
    if (n < 0 || n > PN_MAX_N || ncomp < 1 || ncomp > kMaxComp || ngrid < 0) return 0;
    const size_t pearson = ((size_t)ncomp * kPart * 3 + (size_t)ncomp * 2) * sizeof(double);
    const size_t kde = (size_t)ncomp * kPart * (size_t)ngrid * sizeof(double);
    return pearson > kde ? pearson : kde;
}

int pn_pearson(int64_t n, int64_t ld, const double* x, const double* y, int32_t ncomp, double* out,
               void* workspace, size_t ws_bytes, void* stream) {
    if (bad_common(n, ld, ncomp) || !out || (n > 0 && (!x || !y))) return PN_EINVAL;
    if (!workspace || ws_bytes < pn_stats_workspace_bytes(n, ncomp, 0)) return PN_EINVAL;
    const int rc = device_ready();
    if (rc != PN_OK) return rc;
    hipStream_t s = (hipStream_t)stream;
    if (n == 0) {
        hipLaunchKernelGGL(fill_nan, dim3(1), dim3(kBlock), 0, s, out, (int)(ncomp * 5));
        return launched();
    }
    double* part = (double*)workspace;
    double* mean = part + (size_t)ncomp * kPart * 3;
    hipLaunchKernelGGL(sums_kernel, dim3(kPart, ncomp), dim3(kBlock), 0, s, n, ld, x, y, part);
    hipLaunchKernelGGL(means_kernel, dim3(ncomp), dim3(kBlock), 0, s, n, part, mean);
    hipLaunchKernelGGL(centred_kernel, dim3(kPart, ncomp), dim3(kBlock), 0, s, n, ld, x, y, mean, part);
    hipLaunchKernelGGL(pearson_final_kernel, dim3(ncomp), dim3(kBlock), 0, s, n, part, mean, out);
    return launched();
}

int pn_kde(int64_t n, int64_t ld, const double* x, int32_t ncomp, const double* sigma, int64_t sigma_stride,
           int32_t ngrid, double lo, double hi, double* out, void* workspace, size_t ws_bytes, void* stream) {
    if (bad_common(n, ld, ncomp) || ngrid < 2 || ngrid > 4096 || !(lo < hi) || !std::isfinite(lo) ||
        !std::isfinite(hi) || !out || !sigma || sigma_stride < 1 || (n > 0 && !x))
        return PN_EINVAL;
    if (!workspace || ws_bytes < pn_stats_workspace_bytes(n, ncomp, ngrid)) return PN_EINVAL;
    const int rc = device_ready();
    if (rc != PN_OK) return rc;
    hipStream_t s = (hipStream_t)stream;
    if (n == 0) {
        hipLaunchKernelGGL(fill_nan, dim3((ncomp * ngrid + kBlock - 1) / kBlock), dim3(kBlock), 0, s, out,
                           (int)(ncomp * ngrid));
        return launched();
    }
    const double nfac = std::pow((double)n, -0.2);
    const double gstep = (hi - lo) / (ngrid - 1);
    const double sqrt2pi = std::sqrt(2.0 * 3.14159265358979323846);
    double* part = (double*)workspace;
    hipLaunchKernelGGL(kde_kernel, dim3(kPart, ncomp), dim3(kBlock), 0, s, n, ld, x, sigma, sigma_stride, nfac,
                       (int)ngrid, lo, gstep, part);
    hipLaunchKernelGGL(kde_final_kernel, dim3((ngrid + kBlock - 1) / kBlock, ncomp), dim3(kBlock), 0, s, n, sigma,
                       sigma_stride, nfac, sqrt2pi, (int)ngrid, part, out);
    return launched();
}

size_t pn_ks_workspace_bytes(int64_t n) {
    if (n < 0 || n > PN_MAX_N) return 0;
    const size_t tmp = radix_temp_bytes(n);
    if (n > 0 && tmp == 0) return 0;
    // sorted copy, sort scratch (256-byte aligned), partial maxima
    return ((size_t)n * sizeof(double) + 255) / 256 * 256 + (tmp + 255) / 256 * 256 + kPart * sizeof(double);
}

int pn_ks_uniform(int64_t n, int64_t ld, const double* x, int32_t ncomp, double lo, double hi, double* out,
                  void* workspace, size_t ws_bytes, void* stream) {
    if (bad_common(n, ld, ncomp) || !(lo < hi) || !std::isfinite(lo) || !std::isfinite(hi) || !out ||
        (n > 0 && !x))
        return PN_EINVAL;
    const int rc = device_ready();
    if (rc != PN_OK) return rc;
    hipStream_t s = (hipStream_t)stream;
    if (n == 0) {
        hipLaunchKernelGGL(fill_nan, dim3(1), dim3(kBlock), 0, s, out, (int)(ncomp * 2));
        return launched();
    }
    const size_t need = pn_ks_workspace_bytes(n);
    if (need == 0 || !workspace || ws_bytes < need) return PN_EINVAL;
    char* w = (char*)workspace;
    double* sorted = (double*)w;
    size_t off = ((size_t)n * sizeof(double) + 255) / 256 * 256;
    void* tmp = w + off;
    size_t tmp_bytes = radix_temp_bytes(n);
    off += (tmp_bytes + 255) / 256 * 256;
    double* part = (double*)(w + off);
    for (int c = 0; c < ncomp; ++c) {
        if (rocprim::radix_sort_keys(tmp, tmp_bytes, x + (int64_t)c * ld, sorted, (size_t)n, 0, 64, s) != hipSuccess)
            return PN_EHIP;
        hipLaunchKernelGGL(ks_kernel, dim3(kPart), dim3(kBlock), 0, s, n, sorted, lo, hi, part);
        hipLaunchKernelGGL(ks_final_kernel, dim3(1), dim3(64), 0, s, n, part, out + 2 * c);
    }
    return launched();
}

}  // extern "C"
