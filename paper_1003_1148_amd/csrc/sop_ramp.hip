// The exactly solvable model of Section IV.C that measures the accuracy of
// the integrators: an ensemble of independent Brownian particles X in the
// harmonic well K_sp X^2/2 pulled by the force ramp r_f t, advanced by the
// first-order scheme (Eq. 2, whose mean obeys Eq. 4) or the second-order
// one (whose mean obeys Eq. 5), with single-precision positions held either
// as a compensated pair (hi, lo) or as plain floats.  The ensemble moments
// are summed in double precision in a fixed order.
#include <cmath>
#include <mutex>

#include "sop_internal.hpp"
#include "sop_rng.hpp"

namespace sop {
namespace {

constexpr int RAMP_WG = 256;
constexpr int RAMP_MAX_BLOCKS = 1024;  // blocks of the moment reduction

struct RampConsts {
    double rf_h;      // r_f h: the ramp force at step k is k r_f h
    float k_sp;
    float c_det;      // h/xi (order 1) or (h/xi)(1 - h/(2 tau)) (order 2)
    float c_noise;    // sqrt(2 kB T h/xi)
    unsigned key0, key1, stream;
};

// Both schemes step X by c_det (r_f t_k - K_sp X) plus the Gaussian
// displacement: the order-2 correction of Eq. 5,
// (X/(2 tau^2) - r_f t_k/(2 tau xi)) h^2, is -(h/(2 tau)) times the order-1
// drift (r_f t_k/xi - X/tau) h, so it only rescales the drift coefficient.
template <bool COMP, bool NOISE>
__global__ __launch_bounds__(RAMP_WG) void k_ramp(float2 *__restrict__ x, long long m_count,
                                                  long long step0, long long n_steps, RampConsts c)
{
    const long long m = (long long)blockIdx.x * RAMP_WG + threadIdx.x;
    if (m >= m_count)
        return;
    float2 v = x[m];
    float hi = v.x, lo = COMP ? v.y : 0.0f;
    for (long long k = step0; k < step0 + n_steps; ++k) {
        // the ramp force in double (k reaches 1e9 and more), the rest single
        const float ramp = (float)(c.rf_h * (double)k);
        const float f = (ramp - c.k_sp * hi) - c.k_sp * lo;
        float delta = c.c_det * f;
        if (NOISE) {
            const uint4 w = philox10(make_uint4((unsigned)m, c.stream, (unsigned)k,
                                                (unsigned)((unsigned long long)k >> 32)),
                                     c.key0, c.key1);
            delta += c.c_noise * gaussian_pair(w).x;
        }
        if (COMP) {
            // TwoSum(hi, delta + lo): hi + lo keeps the increments that fall
            // below half an ulp of hi
            const float y = delta + lo;
            const float t = hi + y;
            const float bp = t - hi;
            const float ap = t - bp;
            lo = (hi - ap) + (y - bp);
            hi = t;
        } else {
            hi = hi + delta;
        }
    }
    x[m] = make_float2(hi, lo);
}

// Per-block double sums of X = hi + lo and X^2 over a grid-stride range.
__global__ __launch_bounds__(RAMP_WG) void k_ramp_partial(const float2 *__restrict__ x, long long m_count,
                                                          double *__restrict__ part)
{
    __shared__ double s1[RAMP_WG], s2[RAMP_WG];
    double a = 0.0, b = 0.0;
    for (long long m = (long long)blockIdx.x * RAMP_WG + threadIdx.x; m < m_count;
         m += (long long)gridDim.x * RAMP_WG) {
        const float2 v = x[m];
        const double X = (double)v.x + (double)v.y;
        a += X;
        b += X * X;
    }
    s1[threadIdx.x] = a;
    s2[threadIdx.x] = b;
    __syncthreads();
    for (int off = RAMP_WG / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) {
            s1[threadIdx.x] += s1[threadIdx.x + off];
            s2[threadIdx.x] += s2[threadIdx.x + off];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = s1[0];
        part[2 * blockIdx.x + 1] = s2[0];
    }
}

// Mean and population variance from the block sums, in block order.
__global__ void k_ramp_final(const double *__restrict__ part, int n_part, long long m_count,
                             double *__restrict__ moments)
{
    if (threadIdx.x != 0 || blockIdx.x != 0)
        return;
    double a = 0.0, b = 0.0;
    for (int k = 0; k < n_part; ++k) {
        a += part[2 * k];
        b += part[2 * k + 1];
    }
    const double mean = a / (double)m_count;
    moments[0] = mean;
    moments[1] = b / (double)m_count - mean * mean;
}

int ramp_blocks(long long m_count)
{
    const long long b = (m_count + RAMP_WG - 1) / RAMP_WG;
    return (int)std::max<long long>(1, std::min<long long>(b, RAMP_MAX_BLOCKS));
}

sop_status ramp_check(const sop_ramp_params *rp, int64_t n_particles, const float *x, int64_t step0,
                      int64_t n_steps)
{
    if (!rp || !x || n_particles < 1 || n_particles > INT32_MAX || step0 < 0 || n_steps < 0)
        return SOP_E_ARG;
    if (rp->order != 1 && rp->order != 2)
        return SOP_E_ARG;
    if (!(rp->xi > 0.0) || !(rp->k_sp >= 0.0) || !(rp->kBT >= 0.0) || !(rp->h > 0.0) ||
        !std::isfinite(rp->rf))
        return SOP_E_ARG;
    return SOP_OK;
}

// The steps and the moments, with the block sums in `part`
// (2 * RAMP_MAX_BLOCKS doubles of device memory).
sop_status ramp_launch(const sop_ramp_params *rp, int64_t n_particles, float *x, int64_t step0,
                       int64_t n_steps, double *part, double *moments, hipStream_t s)
{
    RampConsts c;
    c.rf_h = rp->rf * rp->h;
    c.k_sp = (float)rp->k_sp;
    const double tau_inv = rp->k_sp / rp->xi;
    const double cd = rp->h / rp->xi * (rp->order == 2 ? 1.0 - 0.5 * rp->h * tau_inv : 1.0);
    c.c_det = (float)cd;
    c.c_noise = (float)std::sqrt(2.0 * rp->kBT * rp->h / rp->xi);
    c.key0 = (unsigned)(rp->seed & 0xffffffffu);
    c.key1 = (unsigned)(rp->seed >> 32);
    c.stream = rp->stream;
    float2 *xv = reinterpret_cast<float2 *>(x);
    const long long M = n_particles;
    const int grid = (int)((M + RAMP_WG - 1) / RAMP_WG);
    const bool noise = rp->kBT > 0.0;
    if (n_steps > 0) {
        if (rp->compensated)
            noise ? k_ramp<true, true><<<grid, RAMP_WG, 0, s>>>(xv, M, step0, n_steps, c)
                  : k_ramp<true, false><<<grid, RAMP_WG, 0, s>>>(xv, M, step0, n_steps, c);
        else
            noise ? k_ramp<false, true><<<grid, RAMP_WG, 0, s>>>(xv, M, step0, n_steps, c)
                  : k_ramp<false, false><<<grid, RAMP_WG, 0, s>>>(xv, M, step0, n_steps, c);
    }
    if (moments) {
        const int nb = ramp_blocks(M);
        k_ramp_partial<<<nb, RAMP_WG, 0, s>>>(xv, M, part);
        k_ramp_final<<<1, 64, 0, s>>>(part, nb, M, moments);
    }
    return hipGetLastError() == hipSuccess ? SOP_OK : SOP_E_HIP;
}

// Fixed scratch of the allocation-free entry point: the block sums of the
// moment reduction (at most RAMP_MAX_BLOCKS blocks whatever the particle
// count).  One copy per GPU, at its own device address.
static __device__ __align__(256) double scratch[2 * RAMP_MAX_BLOCKS];

constexpr int MAX_DEVICES = 64;
std::mutex scratch_mu;
double *scratch_ptr[MAX_DEVICES] = {};

// The current device's address of `scratch`, looked up once per device.
sop_status scratch_on_current_device(double **out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES)
        return SOP_E_HIP;
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p)
            return SOP_E_HIP;
        scratch_ptr[dev] = static_cast<double *>(p);
    }
    *out = scratch_ptr[dev];
    return SOP_OK;
}

}  // namespace
}  // namespace sop

using namespace sop;

extern "C" {

sop_status sop_ramp_workspace_size(int64_t n_particles, size_t *bytes)
{
    if (!bytes || n_particles < 1)
        return SOP_E_ARG;
    *bytes = (size_t)2 * ramp_blocks(n_particles) * sizeof(double);
    return SOP_OK;
}

sop_status sop_ramp_run(const sop_ramp_params *rp, int64_t n_particles, float *x, int64_t step0,
                        int64_t n_steps, void *workspace, size_t workspace_bytes, double *moments,
                        void *hip_stream)
{
    sop_status st = ramp_check(rp, n_particles, x, step0, n_steps);
    if (st != SOP_OK)
        return st;
    if (moments) {
        size_t need = 0;
        sop_ramp_workspace_size(n_particles, &need);
        if (!workspace || workspace_bytes < need || ((uintptr_t)workspace & 7u))
            return SOP_E_WORKSPACE;
    }
    return ramp_launch(rp, n_particles, x, step0, n_steps, static_cast<double *>(workspace), moments,
                       static_cast<hipStream_t>(hip_stream));
}

sop_status sop_ramp_run_static(const sop_ramp_params *rp, int64_t n_particles, float *x, int64_t step0,
                               int64_t n_steps, double *moments, void *hip_stream)
{
    sop_status st = ramp_check(rp, n_particles, x, step0, n_steps);
    if (st != SOP_OK)
        return st;
    double *part = nullptr;
    if (moments) {
        st = scratch_on_current_device(&part);
        if (st != SOP_OK)
            return st;
    }
    return ramp_launch(rp, n_particles, x, step0, n_steps, part, moments,
                       static_cast<hipStream_t>(hip_stream));
}

}  // extern "C"
