// Time stepping around the force (Section 2.2 kicks the velocities with the forces and then
// drifts the positions; Section 2.4 eq. (7) gives the shared step).  FP64 without contraction,
// so each value is the plain IEEE evaluation of the formula.
//  * k_timestep: min over particles of sqrt(eps / |a_i|) and eps / |v_i| (a zero denominator
//    does not bind); positive doubles order like their bit patterns, so the minimum is an
//    integer atomicMin and does not depend on the order of the blocks;
//  * k_kick_drift: v += a dt_kick, then x += v dt_drift, wrapped back into [0, L).
#include "common.hpp"

#include <mutex>

// Scratch of treepm_timestep_noalloc: the reduction word, in static device memory so that the
// call allocates nothing.  Each GPU the library runs on holds its own copy until the process
// ends; every call on one GPU shares it (calls that overlap on one GPU race).  Host code must
// not pass this name to a kernel: it is a host-side stand-in, and the device address comes
// from hipGetSymbolAddress (step_scratch below).
static __device__ __align__(256) unsigned long long scratch[tpm::kStepScratchWords];

namespace tpm {
namespace {

template <typename A>
__global__ __launch_bounds__(256) void k_timestep(int64_t n, const double *__restrict__ vx,
                                                  const double *__restrict__ vy,
                                                  const double *__restrict__ vz,
                                                  const A *__restrict__ ax,
                                                  const A *__restrict__ ay,
                                                  const A *__restrict__ az, double eps,
                                                  unsigned long long *out)
{
    unsigned long long best = 0x7ff0000000000000ull; // +inf
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double a0 = ax[i], a1 = ay[i], a2 = az[i];
        const double v0 = vx[i], v1 = vy[i], v2 = vz[i];
        const double am = sqrt(a0 * a0 + a1 * a1 + a2 * a2);
        const double vm = sqrt(v0 * v0 + v1 * v1 + v2 * v2);
        if (am > 0.0) {
            const unsigned long long t = (unsigned long long)__double_as_longlong(sqrt(eps / am));
            best = t < best ? t : best;
        }
        if (vm > 0.0) {
            const unsigned long long t = (unsigned long long)__double_as_longlong(eps / vm);
            best = t < best ? t : best;
        }
    }
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) {
        const unsigned long long o = __shfl_xor(best, d, 64);
        best = o < best ? o : best;
    }
    if ((threadIdx.x & 63) == 0) atomicMin(out, best);
}

template <typename A>
__global__ __launch_bounds__(256) void k_kick_drift(int64_t n, double *__restrict__ x,
                                                    double *__restrict__ y,
                                                    double *__restrict__ z,
                                                    double *__restrict__ vx,
                                                    double *__restrict__ vy,
                                                    double *__restrict__ vz,
                                                    const A *__restrict__ ax,
                                                    const A *__restrict__ ay,
                                                    const A *__restrict__ az, double dt_kick,
                                                    double dt_drift, double L)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    double *const pos[3] = {x, y, z};
    double *const vel[3] = {vx, vy, vz};
    const A *const acc[3] = {ax, ay, az};
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const double v = vel[c][i] + (double)acc[c][i] * dt_kick;
        double p = pos[c][i] + v * dt_drift;
        if (p >= L) p -= L;
        if (p < 0.0) p += L;
        if (p >= L) p = 0.0; // just below 0, rounded to L when L was added
        vel[c][i] = v;
        pos[c][i] = p;
    }
}

} // namespace

void launch_timestep(int64_t n, const double *vx, const double *vy, const double *vz,
                     const void *ax, const void *ay, const void *az, int acc_fp64, double eps,
                     unsigned long long *out, hipStream_t s)
{
    fill_u64((uint64_t *)out, 1, 0x7ff0000000000000ull, s);
    if (!n) return;
    const int64_t b = (n + 255) / 256;
    const unsigned g = (unsigned)(b < 2048 ? b : 2048);
    if (acc_fp64)
        k_timestep<double><<<g, 256, 0, s>>>(n, vx, vy, vz, (const double *)ax,
                                             (const double *)ay, (const double *)az, eps, out);
    else
        k_timestep<float><<<g, 256, 0, s>>>(n, vx, vy, vz, (const float *)ax,
                                            (const float *)ay, (const float *)az, eps, out);
}

hipError_t step_scratch(int device, unsigned long long **out)
{
    static std::mutex mu;
    static unsigned long long *ptr[kMaxDevices] = {};
    *out = nullptr;
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(mu);
    if (!ptr[device]) {
        // the caller has made `device` current: this is that device's copy of the array
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        ptr[device] = static_cast<unsigned long long *>(p);
    }
    *out = ptr[device];
    return hipSuccess;
}

void launch_kick_drift(int64_t n, double *x, double *y, double *z, double *vx, double *vy,
                       double *vz, const void *ax, const void *ay, const void *az, int acc_fp64,
                       double dt_kick, double dt_drift, double L, hipStream_t s)
{
    if (!n) return;
    const unsigned b = (unsigned)((n + 255) / 256);
    if (acc_fp64)
        k_kick_drift<double><<<b, 256, 0, s>>>(n, x, y, z, vx, vy, vz, (const double *)ax,
                                               (const double *)ay, (const double *)az, dt_kick,
                                               dt_drift, L);
    else
        k_kick_drift<float><<<b, 256, 0, s>>>(n, x, y, z, vx, vy, vz, (const float *)ax,
                                              (const float *)ay, (const float *)az, dt_kick,
                                              dt_drift, L);
}

} // namespace tpm
