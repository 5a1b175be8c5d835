// Short-range pair force over the interaction lists (Section 2.1 eq. 1 with the cutoff
// g_P3M of eq. 2 and Plummer softening of Section 2.4):
//
//   a_i += m_j d g(|d| / eta) / (|d|^2 + eps^2)^(3/2),   d = x_j - x_i.
//
// One 64-lane wavefront per group: each lane holds one i-particle (groups larger than 64 are
// done in chunks of 64), and the group's list is streamed through LDS in tiles; every lane
// reads the same tile entry (an LDS broadcast) and accumulates into registers.
//
// FP32 path (Section 3.1.1): positions are passed relative to the group's cube centre x_g,
// x_i - x_g and wrap(x_j - x_g), each difference taken in FP64 and then rounded to FP32, so
// the rounding error of the subtraction scales with the group size, not the box.  The
// per-tile FP32 partial sums are folded into an FP32 (hi, lo) pair with TwoSum.
//
// FP64 path: plain FP64 on absolute positions with the nearest image per pair, IEEE square
// root and division.
//
// g is evaluated in a form with no cancellation: for R < 1,
//   g = 1 + R^3 (-8/5 + R^2 (8/5 + R (-1/2 + R (-12/35 + 3R/20)))),
// and for R >= 1, g = max(2 - R, 0)^5 (7R^3 + 22R^2 + 10R + 4) / 140 (zero from R = 2 on).
// Both are eq. (2) rearranged.
#include "common.hpp"

namespace tpm {
namespace {

constexpr int kTileJ = 64;

__device__ __forceinline__ float g_p3m_f32(float R)
{
    float R2 = R * R;
    float p = fmaf(0.15f, R, -12.0f / 35.0f);
    p = fmaf(p, R, -0.5f);
    p = fmaf(p, R, 1.6f);
    p = fmaf(p, R2, -1.6f);
    float g1 = fmaf(p, R2 * R, 1.0f);
    float u = fmaxf(2.0f - R, 0.0f);
    float u2 = u * u;
    float u5 = u2 * u2 * u;
    float c = fmaf(fmaf(fmaf(0.05f, R, 22.0f / 140.0f), R, 10.0f / 140.0f), R, 4.0f / 140.0f);
    float g2 = u5 * c;
    return R < 1.0f ? g1 : g2;
}

__device__ __forceinline__ double g_p3m_f64(double R)
{
    double R2 = R * R;
    double p = fma(0.15, R, -12.0 / 35.0);
    p = fma(p, R, -0.5);
    p = fma(p, R, 1.6);
    p = fma(p, R2, -1.6);
    double g1 = fma(p, R2 * R, 1.0);
    double u = fmax(2.0 - R, 0.0);
    double u2 = u * u;
    double u5 = u2 * u2 * u;
    double c = fma(fma(fma(0.05, R, 22.0 / 140.0), R, 10.0 / 140.0), R, 4.0 / 140.0);
    return R < 1.0 ? g1 : u5 * c;
}

__device__ __forceinline__ double wrapd(double v, double L)
{
    double h = 0.5 * L;
    if (v >= h) return v - L;
    if (v < -h) return v + L;
    return v;
}

__device__ __forceinline__ void two_sum_fold(float &hi, float &lo, float t)
{
    float s = hi + t;
    float bp = s - hi;
    float err = (hi - (s - bp)) + (t - bp);
    hi = s;
    lo += err;
}

template <int OUT64>
__device__ __forceinline__ void store3(void *ax, void *ay, void *az, uint32_t i, double vx,
                                       double vy, double vz)
{
    if (OUT64) {
        ((double *)ax)[i] = vx;
        ((double *)ay)[i] = vy;
        ((double *)az)[i] = vz;
    } else {
        ((float *)ax)[i] = (float)vx;
        ((float *)ay)[i] = (float)vy;
        ((float *)az)[i] = (float)vz;
    }
}

template <int OUT64>
__global__ __launch_bounds__(64) void k_force_f32(
    NodeArrays nd, GroupArrays gr, uint32_t n_groups, const uint64_t *__restrict__ off,
    const uint32_t *__restrict__ entries, const double *__restrict__ px,
    const double *__restrict__ py, const double *__restrict__ pz, const double *__restrict__ pm,
    const uint32_t *__restrict__ pidx, ForceParams fp, void *ax, void *ay, void *az)
{
    __shared__ float4 tile[kTileJ];
    const uint32_t g = blockIdx.x;
    const int lane = threadIdx.x;
    if (g >= n_groups) return;
    const uint32_t n_g = gr.count[g], f = gr.first[g];
    const uint64_t b = off[g];
    const uint64_t Lg = off[g + 1] - b;
    const double xg0 = gr.xgx[g], xg1 = gr.xgy[g], xg2 = gr.xgz[g];
    const double L = fp.L;
    const float eps2 = (float)fp.eps2, inv_eta = (float)fp.inv_eta;
    for (uint32_t ib = 0; ib < n_g; ib += 64) {
        const uint32_t i = ib + lane;
        const bool act = i < n_g;
        float xi = 0.f, yi = 0.f, zi = 0.f;
        if (act) {
            xi = (float)(px[f + i] - xg0);
            yi = (float)(py[f + i] - xg1);
            zi = (float)(pz[f + i] - xg2);
        }
        float hx = 0.f, hy = 0.f, hz = 0.f, lx = 0.f, ly = 0.f, lz = 0.f;
        for (uint64_t jb = 0; jb < Lg; jb += kTileJ) {
            const uint64_t j = jb + lane;
            float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
            if (j < Lg) {
                uint32_t e = entries[b + j];
                double sx, sy, sz, sm;
                if (e & kCellTag) {
                    uint32_t u = e & ~kCellTag;
                    sx = nd.comx[u]; sy = nd.comy[u]; sz = nd.comz[u]; sm = nd.mass[u];
                } else {
                    sx = px[e]; sy = py[e]; sz = pz[e]; sm = pm[e];
                }
                v = make_float4((float)wrapd(sx - xg0, L), (float)wrapd(sy - xg1, L),
                                (float)wrapd(sz - xg2, L), (float)sm);
            }
            tile[lane] = v;
            __syncthreads();
            const int nt = (Lg - jb) < (uint64_t)kTileJ ? (int)(Lg - jb) : kTileJ;
            float tx = 0.f, ty = 0.f, tz = 0.f;
            for (int t = 0; t < nt; ++t) {
                const float4 s = tile[t];
                const float dx = s.x - xi, dy = s.y - yi, dz = s.z - zi;
                const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
                const float rinv = __builtin_amdgcn_rsqf(r2 + eps2);
                const float rinv3 = rinv * rinv * rinv;
                const float R = __builtin_amdgcn_sqrtf(r2) * inv_eta;
                const float fm = s.w * g_p3m_f32(R) * rinv3;
                tx = fmaf(fm, dx, tx);
                ty = fmaf(fm, dy, ty);
                tz = fmaf(fm, dz, tz);
            }
            __syncthreads();
            two_sum_fold(hx, lx, tx);
            two_sum_fold(hy, ly, ty);
            two_sum_fold(hz, lz, tz);
        }
        if (act)
            store3<OUT64>(ax, ay, az, pidx[f + i], (double)hx + (double)lx,
                          (double)hy + (double)ly, (double)hz + (double)lz);
    }
}

struct d4 {
    double x, y, z, m;
};

template <int OUT64>
__global__ __launch_bounds__(64) void k_force_f64(
    NodeArrays nd, GroupArrays gr, uint32_t n_groups, const uint64_t *__restrict__ off,
    const uint32_t *__restrict__ entries, const double *__restrict__ px,
    const double *__restrict__ py, const double *__restrict__ pz, const double *__restrict__ pm,
    const uint32_t *__restrict__ pidx, ForceParams fp, void *ax, void *ay, void *az)
{
    __shared__ d4 tile[kTileJ];
    const uint32_t g = blockIdx.x;
    const int lane = threadIdx.x;
    if (g >= n_groups) return;
    const uint32_t n_g = gr.count[g], f = gr.first[g];
    const uint64_t b = off[g];
    const uint64_t Lg = off[g + 1] - b;
    const double L = fp.L, eps2 = fp.eps2, eta = fp.eta;
    for (uint32_t ib = 0; ib < n_g; ib += 64) {
        const uint32_t i = ib + lane;
        const bool act = i < n_g;
        double xi = 0.0, yi = 0.0, zi = 0.0;
        if (act) {
            xi = px[f + i];
            yi = py[f + i];
            zi = pz[f + i];
        }
        double ax_ = 0.0, ay_ = 0.0, az_ = 0.0;
        for (uint64_t jb = 0; jb < Lg; jb += kTileJ) {
            const uint64_t j = jb + lane;
            d4 v = {0.0, 0.0, 0.0, 0.0};
            if (j < Lg) {
                uint32_t e = entries[b + j];
                if (e & kCellTag) {
                    uint32_t u = e & ~kCellTag;
                    v = {nd.comx[u], nd.comy[u], nd.comz[u], nd.mass[u]};
                } else {
                    v = {px[e], py[e], pz[e], pm[e]};
                }
            }
            tile[lane] = v;
            __syncthreads();
            const int nt = (Lg - jb) < (uint64_t)kTileJ ? (int)(Lg - jb) : kTileJ;
            for (int t = 0; t < nt; ++t) {
                const d4 s = tile[t];
                const double dx = wrapd(s.x - xi, L), dy = wrapd(s.y - yi, L),
                             dz = wrapd(s.z - zi, L);
                const double r2 = dx * dx + dy * dy + dz * dz;
                const double r = sqrt(r2);
                const double s2 = r2 + eps2;
                double fm = s.m * g_p3m_f64(r / eta) / (s2 * sqrt(s2));
                fm = r2 > 0.0 ? fm : 0.0;
                ax_ += fm * dx;
                ay_ += fm * dy;
                az_ += fm * dz;
            }
            __syncthreads();
        }
        if (act) store3<OUT64>(ax, ay, az, pidx[f + i], ax_, ay_, az_);
    }
}

} // namespace

void launch_force_f32(NodeArrays nd, GroupArrays gr, uint32_t n_groups, const uint64_t *off,
                      const uint32_t *entries, const double *px, const double *py,
                      const double *pz, const double *pm, const uint32_t *pidx,
                      ForceParams fp, void *ax, void *ay, void *az, int out_prec,
                      hipStream_t s)
{
    if (!n_groups) return;
    if (out_prec)
        k_force_f32<1><<<n_groups, 64, 0, s>>>(nd, gr, n_groups, off, entries, px, py, pz, pm,
                                              pidx, fp, ax, ay, az);
    else
        k_force_f32<0><<<n_groups, 64, 0, s>>>(nd, gr, n_groups, off, entries, px, py, pz, pm,
                                              pidx, fp, ax, ay, az);
}

void launch_force_f64(NodeArrays nd, GroupArrays gr, uint32_t n_groups, const uint64_t *off,
                      const uint32_t *entries, const double *px, const double *py,
                      const double *pz, const double *pm, const uint32_t *pidx,
                      ForceParams fp, void *ax, void *ay, void *az, int out_prec,
                      hipStream_t s)
{
    if (!n_groups) return;
    if (out_prec)
        k_force_f64<1><<<n_groups, 64, 0, s>>>(nd, gr, n_groups, off, entries, px, py, pz, pm,
                                              pidx, fp, ax, ay, az);
    else
        k_force_f64<0><<<n_groups, 64, 0, s>>>(nd, gr, n_groups, off, entries, px, py, pz, pm,
                                              pidx, fp, ax, ay, az);
}

} // namespace tpm
