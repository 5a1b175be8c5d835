// Quadrupole term of the cell entries (Section 4.1: the second-order moment of a cell, whose
// expansion must carry the spatial derivatives of the cutoff function).
//
// For a cell of mass M, centre of mass X and second moment Q = sum m s s^T about X, the
// particles' pair law F(d) = d h(r), h = g(r/eta) (r^2 + eps^2)^(-3/2), summed over the cell is,
// to second order in the offsets s,
//     M F(d) + (Q d) u + (1/2) tr(Q) d u + (1/2) (d.Q.d) d w,   u = h'/r,  w = (h'/r)'/r,
// with d = X - x_i.  The force kernels add the first term for every cell entry; this file
// adds the rest, after them, for boxes that ask for it:
//  * k_second_moments: Q per node in FP64, level by level from the leaves up (a leaf from its
//    particles, an internal node from its children by the parallel-axis theorem);
//  * k_quad<T>: one wave per group; its list's cell entries that can reach the group (gap to
//    the group's box < r_cut) are gathered into LDS 64 at a time, and the lanes add their
//    terms to the group's particles' acceleration records (small groups spread each particle's
//    cells over several lanes), in T = float (relative to the group's cube centre, as the
//    FP32 force kernel; hardware reciprocal square roots) or double.
#include "common.hpp"

namespace tpm {
namespace {

constexpr int kQuadTile = 64;

__device__ __forceinline__ double wrapq(double v, double L)
{
    const double h = 0.5 * L;
    if (v >= h) return v - L;
    if (v < -h) return v + L;
    return v;
}

__global__ __launch_bounds__(256) void k_second_moments(NodeArrays nd,
                                                        const double4 *__restrict__ ps,
                                                        uint32_t lo, uint32_t hi,
                                                        double *__restrict__ Q)
{
    for (uint32_t u = lo + blockIdx.x * blockDim.x + threadIdx.x; u < hi;
         u += gridDim.x * blockDim.x) {
        const double4 cu = nd.nsrc[u]; // centre of mass, mass
        const double X = cu.x, Y = cu.y, Z = cu.z;
        double q[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        const uint32_t nch = nd.nchild[u];
        if (nch == 0) {
            const uint32_t f = nd.first[u], e = f + nd.count[u];
            for (uint32_t k = f; k < e; ++k) {
                const double4 r = ps[k];
                const double dx = r.x - X, dy = r.y - Y, dz = r.z - Z;
                q[0] += r.w * dx * dx;
                q[1] += r.w * dy * dy;
                q[2] += r.w * dz * dz;
                q[3] += r.w * dx * dy;
                q[4] += r.w * dx * dz;
                q[5] += r.w * dy * dz;
            }
        } else {
            const uint32_t cf = nd.child_first[u];
            for (uint32_t c = cf; c < cf + nch; ++c) {
                const double4 cc = nd.nsrc[c];
                const double m = cc.w;
                const double dx = cc.x - X, dy = cc.y - Y, dz = cc.z - Z;
                const double *qc = Q + 6 * (size_t)c;
                q[0] += qc[0] + m * dx * dx;
                q[1] += qc[1] + m * dy * dy;
                q[2] += qc[2] + m * dz * dz;
                q[3] += qc[3] + m * dx * dy;
                q[4] += qc[4] + m * dx * dz;
                q[5] += qc[5] + m * dy * dz;
            }
        }
        for (int a = 0; a < 6; ++a) Q[6 * (size_t)u + a] = q[a];
    }
}

// g(R) of eq. (2) and its first two derivatives, each times 140: the expanded first branch,
// and the second branch as (2 - R)^5 P(R), P = 7R^3 + 22R^2 + 10R + 4, differentiated as a
// product so that nothing cancels near R = 2.
template <typename T>
__device__ __forceinline__ void g_derivs140(T R, T &g, T &g1, T &g2)
{
    if (R < T(1)) {
        const T R2 = R * R;
        g = T(140) - R2 * R * (T(224) + R2 * (T(-224) + R * (T(70) + R * (T(48) - T(21) * R))));
        g1 = -R2 * (T(672) + R2 * (T(-1120) + R * (T(420) + R * (T(336) - T(168) * R))));
        g2 = -R * (T(1344) + R2 * (T(-4480) + R * (T(2100) + R * (T(2016) - T(1176) * R))));
    } else if (R < T(2)) {
        const T v = T(2) - R, v2 = v * v, v3 = v2 * v;
        const T P = T(4) + R * (T(10) + R * (T(22) + T(7) * R));
        const T P1 = T(10) + R * (T(44) + T(21) * R);
        const T P2 = T(44) + T(42) * R;
        g = v3 * v2 * P;
        g1 = v3 * v * (v * P1 - T(5) * P);
        g2 = v3 * (T(20) * P - T(10) * v * P1 + v2 * P2);
    } else {
        g = g1 = g2 = T(0);
    }
}

// The second branch alone, for pairs known to have R >= 1 (clamped to zero from R = 2 on).
template <typename T>
__device__ __forceinline__ void g_derivs140_far(T R, T &g, T &g1, T &g2)
{
    const T v = R < T(2) ? T(2) - R : T(0), v2 = v * v, v3 = v2 * v;
    const T P = T(4) + R * (T(10) + R * (T(22) + T(7) * R));
    const T P1 = T(10) + R * (T(44) + T(21) * R);
    const T P2 = T(44) + T(42) * R;
    g = v3 * v2 * P;
    g1 = v3 * v * (v * P1 - T(5) * P);
    g2 = v3 * (T(20) * P - T(10) * v * P1 + v2 * P2);
}

__device__ __forceinline__ float rsqrt_t(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double rsqrt_t(double x) { return 1.0 / sqrt(x); }

// A cell as the kernel uses it: centre of mass relative to the group's cube centre, half the
// trace of the moments, and the six moments, in the arithmetic type (three 16-byte LDS reads
// in FP32).
template <typename T>
struct alignas(4 * sizeof(T)) QuadCell {
    T x, y, z, htr, q0, q1, q2, q3, q4, q5, pad0, pad1;
};

// One wave per group.  The lanes are S = 64 / J particle slots times J cell phases, J the
// largest power of two with n_g J <= 64 kQuadK: lane (slot, phase) takes up to kQuadK particles
// (slot, slot + S, ...) and every J-th cell of each tile, so a cell read from LDS serves
// several particles and small groups still fill the wave.  The J partial sums of a particle
// are added with lane shuffles at the end.
constexpr int kQuadK = 4;

template <typename T, int REC64, int WRAP>
__global__ __launch_bounds__(64) void k_quad(NodeArrays nd, GroupArrays gr, uint32_t n_groups,
                                             const uint64_t *__restrict__ off,
                                             const uint32_t *__restrict__ len,
                                             const uint32_t *__restrict__ entries,
                                             const double4 *__restrict__ ps,
                                             const uint32_t *__restrict__ pidx,
                                             const double *__restrict__ Q, ForceParams fp,
                                             void *rec)
{
    __shared__ QuadCell<T> tile[kQuadTile];
    const uint32_t g = xcd_block(blockIdx.x, gridDim.x);
    const int lane = threadIdx.x;
    if (g >= n_groups) return;
    const uint32_t n_g = gr.count[g], f = gr.first[g];
    const uint64_t b = off[g], Lg = len[g];
    const double L = fp.L;
    const double xg0 = gr.xgx[g], xg1 = gr.xgy[g], xg2 = gr.xgz[g];
    const double cg0 = gr.cgx[g], cg1 = gr.cgy[g], cg2 = gr.cgz[g];
    const double hg0 = gr.hgx[g], hg1 = gr.hgy[g], hg2 = gr.hgz[g];
    const double half_side = 0.5 * ldexp(L, -(int)nd.level[gr.node[g]]);
    // one image per entry (relative to the cube centre) serves every particle of the group
    // unless half the group cube plus r_cut reaches L/2; then each pair takes its own (only
    // the FP64 path: the FP32 force call refuses such boxes)
    const bool pair_wrap = WRAP && !(half_side + sqrt(fp.rc2) < 0.5 * L);
    const T inv_eta = T(fp.inv_eta), eps2 = T(fp.eps2);
    const T inv_eta2 = inv_eta * inv_eta;
    int lj = 0; // log2 J
    while (lj < 6 && (uint64_t)n_g << (lj + 1) <= 64u * kQuadK) ++lj;
    const int J = 1 << lj, S = 64 >> lj;
    const int slot = lane & (S - 1), ph = lane >> (6 - lj);
    const uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;
    for (uint32_t ib = 0; ib < n_g; ib += (uint32_t)S * kQuadK) {
        T xi[kQuadK], yi[kQuadK], zi[kQuadK], ax_[kQuadK], ay_[kQuadK], az_[kQuadK];
#pragma unroll
        for (int k = 0; k < kQuadK; ++k) {
            const uint32_t i = ib + slot + k * S;
            xi[k] = yi[k] = zi[k] = T(0);
            ax_[k] = ay_[k] = az_[k] = T(0);
            if (i < n_g) {
                const double4 r = ps[f + i];
                xi[k] = T(wrapq(r.x - xg0, L));
                yi[k] = T(wrapq(r.y - xg1, L));
                zi[k] = T(wrapq(r.z - xg2, L));
            }
        }
        // particles this wave holds in the block: how many of the kQuadK slots are used
        const uint32_t rest = n_g - ib;
        const int kk = rest >= (uint32_t)S * kQuadK ? kQuadK : (int)((rest + S - 1) / S);
        for (uint64_t jb = 0; jb < Lg; jb += 64) {
            const uint64_t j = jb + lane;
            bool keep = false, far = false;
            QuadCell<T> v{};
            if (j < Lg) {
                const uint32_t e = entries[b + j];
                if (e & kCellTag) {
                    const uint32_t c = e & ~kCellTag;
                    const double4 r = nd.nsrc[c];
                    double w0 = fabs(wrapq(r.x - cg0, L)) - hg0;
                    double w1 = fabs(wrapq(r.y - cg1, L)) - hg1;
                    double w2 = fabs(wrapq(r.z - cg2, L)) - hg2;
                    w0 = w0 > 0.0 ? w0 : 0.0;
                    w1 = w1 > 0.0 ? w1 : 0.0;
                    w2 = w2 > 0.0 ? w2 : 0.0;
                    const double gap2 = w0 * w0 + w1 * w1 + w2 * w2;
                    keep = gap2 < fp.rc2;
                    far = gap2 >= fp.eta * fp.eta; // every pair has R >= 1
                    const double *q = Q + 6 * (size_t)c;
                    // the moments carry the 1/140 of g and its derivatives below
                    const double k = 1.0 / 140.0;
                    v = QuadCell<T>{T(wrapq(r.x - xg0, L)),
                                    T(wrapq(r.y - xg1, L)),
                                    T(wrapq(r.z - xg2, L)),
                                    T(0.5 * (q[0] + q[1] + q[2]) * k),
                                    T(q[0] * k),
                                    T(q[1] * k),
                                    T(q[2] * k),
                                    T(q[3] * k),
                                    T(q[4] * k),
                                    T(q[5] * k),
                                    T(0),
                                    T(0)};
                }
            }
            // near cells from the front of the tile, far ones from the back
            const uint64_t mn = __ballot(keep && !far), mf = __ballot(keep && far);
            if (keep) {
                if (far)
                    tile[kQuadTile - 1 - __popcll(mf & lt)] = v;
                else
                    tile[__popcll(mn & lt)] = v;
            }
            const int nn = __popcll(mn), nf = __popcll(mf);
            __syncthreads();
            auto pair = [&](const QuadCell<T> &s, bool far_cell, int k) {
                T dx = s.x - xi[k], dy = s.y - yi[k], dz = s.z - zi[k];
                if (WRAP && pair_wrap) {
                    dx = T(wrapq(double(dx), L));
                    dy = T(wrapq(double(dy), L));
                    dz = T(wrapq(double(dz), L));
                }
                // pairs at or beyond r_cut get g = g' = g'' = 0 from the polynomials (R >= 2)
                const T r2 = dx * dx + dy * dy + dz * dz;
                const T ir = r2 > T(0) ? rsqrt_t(r2) : T(0), r = r2 * ir, R = r * inv_eta;
                T gv, g1, g2;
                if (far_cell)
                    g_derivs140_far<T>(R, gv, g1, g2);
                else
                    g_derivs140<T>(R, gv, g1, g2);
                const T is = rsqrt_t(r2 + eps2), is2 = is * is;
                const T q3 = is2 * is, p5 = q3 * is2, s7 = p5 * is2;
                const T ir2 = ir * ir;
                // 140 u = 140 h'/r and 140 w = 140 (h'/r)'/r (the moments carry 1/140)
                const T A = g1 * inv_eta * ir;
                const bool live = r2 > T(0); // a cell never sits on a particle; kept safe
                const T ur = live ? A * q3 - T(3) * gv * p5 : T(0);
                const T wr =
                    live ? (g2 * inv_eta2 - A) * ir2 * q3 - T(6) * A * p5 + T(15) * gv * s7 : T(0);
                const T qx = s.q0 * dx + s.q3 * dy + s.q4 * dz;
                const T qy = s.q3 * dx + s.q1 * dy + s.q5 * dz;
                const T qz = s.q4 * dx + s.q5 * dy + s.q2 * dz;
                const T sc = s.htr * ur + T(0.5) * (dx * qx + dy * qy + dz * qz) * wr;
                ax_[k] += qx * ur + sc * dx;
                ay_[k] += qy * ur + sc * dy;
                az_[k] += qz * ur + sc * dz;
            };
            for (int t = ph; t < nn; t += J) {
                const QuadCell<T> s = tile[t];
#pragma unroll
                for (int k = 0; k < kQuadK; ++k)
                    if (k < kk) pair(s, false, k);
            }
            for (int t = kQuadTile - nf + ph; t < kQuadTile; t += J) {
                const QuadCell<T> s = tile[t];
#pragma unroll
                for (int k = 0; k < kQuadK; ++k)
                    if (k < kk) pair(s, true, k);
            }
            __syncthreads();
        }
        // add the J phases of each particle (lanes slot, slot + S, slot + 2S, ...)
#pragma unroll
        for (int k = 0; k < kQuadK; ++k) {
            for (int d = S; d < 64; d <<= 1) {
                ax_[k] += __shfl_xor(ax_[k], d, 64);
                ay_[k] += __shfl_xor(ay_[k], d, 64);
                az_[k] += __shfl_xor(az_[k], d, 64);
            }
            const uint32_t i = ib + slot + k * S;
            if (i < n_g && ph == 0) {
                const uint32_t o = pidx[f + i];
                if (REC64) {
                    double4 *const r = (double4 *)rec + o;
                    r->x += double(ax_[k]);
                    r->y += double(ay_[k]);
                    r->z += double(az_[k]);
                } else {
                    float4 *const r = (float4 *)rec + o;
                    r->x += float(ax_[k]);
                    r->y += float(ay_[k]);
                    r->z += float(az_[k]);
                }
            }
        }
    }
}

} // namespace

void launch_second_moments(NodeArrays nd, const double4 *ps, uint32_t lo, uint32_t hi,
                           double *Q, hipStream_t s)
{
    if (hi <= lo) return;
    const uint32_t n = hi - lo;
    const uint32_t b = (n + 255) / 256;
    k_second_moments<<<b < 65535 ? b : 65535, 256, 0, s>>>(nd, ps, lo, hi, Q);
}

void launch_quad(NodeArrays nd, GroupArrays gr, uint32_t n_groups, const uint64_t *off,
                 const uint32_t *len, const uint32_t *entries, const double4 *ps,
                 const uint32_t *pidx, const double *Q, ForceParams fp, void *rec,
                 int fp64_math, int rec64, hipStream_t s)
{
    if (!n_groups) return;
    if (fp64_math) {
        if (rec64)
            k_quad<double, 1, 1><<<n_groups, 64, 0, s>>>(nd, gr, n_groups, off, len, entries,
                                                         ps, pidx, Q, fp, rec);
        else
            k_quad<double, 0, 1><<<n_groups, 64, 0, s>>>(nd, gr, n_groups, off, len, entries,
                                                         ps, pidx, Q, fp, rec);
    } else {
        if (rec64)
            k_quad<float, 1, 0><<<n_groups, 64, 0, s>>>(nd, gr, n_groups, off, len, entries,
                                                        ps, pidx, Q, fp, rec);
        else
            k_quad<float, 0, 0><<<n_groups, 64, 0, s>>>(nd, gr, n_groups, off, len, entries,
                                                        ps, pidx, Q, fp, rec);
    }
}

} // namespace tpm
