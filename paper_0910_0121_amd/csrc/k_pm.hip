// Particle-mesh (PM) long-range force on an N^3 periodic mesh (Section 2.2 step 1): TSC
// mass assignment, the potential by FFT with the Green's function of the long-range part of
// the split (the complement of eq. 2), a fourth-order difference for the mesh force and TSC
// interpolation back to the particles.
//
// Mesh layout: point (x, y, z) at (x N + y) N + z, z contiguous; N a power of two.
//  * assignment: a wave sums 256 consecutive particles (key order, so they are close
//    together) into an LDS box of mesh points and adds the box to the mesh; masses are summed
//    as 64-bit fixed point, so the mesh does not depend on the order of the atomics;
//  * FFT: complex, radix 2, one workgroup per bundle of B lines of one axis held in LDS
//    (B N = 4096 values, B <= 16).  Bundles along x and y are B neighbouring lines in z, so a
//    load of one element row is B contiguous values; bundles along z are B contiguous rows.
//    The passes are: x forward (reading the fixed-point masses), y forward, z forward +
//    Green's function + z inverse in one kernel (a DIF forward leaves bit-reversed order, which
//    is what the DIT inverse reads), y inverse, x inverse (writing the real potential);
//  * mesh force: fourth-order central differences of the potential, one float4 per point;
//  * interpolation: one thread per particle (key order) gathers the 27 points of its cloud
//    (neighbouring threads hold neighbouring particles, so the gathers share cache lines) and
//    writes the 16-byte result to the particle's slot in the caller's order through the sort
//    permutation (a scattered write); k_pm_split then writes the three output arrays
//    contiguously.
#include "common.hpp"

namespace tpm {
namespace {

constexpr int kFftThreads = 256;
constexpr int kFftElems = 4096;
constexpr int kMaxTwiddles = 512; // N <= 1024

__device__ __forceinline__ float2 cmul(float2 a, float2 b)
{
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }

// Nearest mesh point of coordinate x for inv_h = N / L.  The product is rounded on its own
// (no contraction into the add), so every kernel finds the same point for the same x.
__device__ __forceinline__ int nearest(double x, double inv_h)
{
#pragma clang fp contract(off)
    return (int)floor(x * inv_h + 0.5);
}

// TSC cloud along one axis: the nearest mesh point (returned) and the weights of the points
// before it, at it and after it.
__device__ __forceinline__ int tsc(double x, double inv_h, double w[3])
{
#pragma clang fp contract(off)
    const double u = x * inv_h;
    const double f = floor(u + 0.5);
    const double d = u - f;
    w[0] = 0.5 * (0.5 - d) * (0.5 - d);
    w[1] = 0.75 - d * d;
    w[2] = 0.5 * (0.5 + d) * (0.5 + d);
    return (int)f;
}

// Fixed-point scale for the mesh masses: a power of two S with n m_max S < 2^62, so no sum
// of contributions can overflow 64 bits.
__device__ __forceinline__ double pm_scale(unsigned long long mmax_bits, int64_t n)
{
    const double t = (double)n * __longlong_as_double((long long)mmax_bits);
    return ldexp(1.0, 61 - ilogb(t));
}

// One wave takes kAssignChunk consecutive particles in key order, kAssignPer consecutive ones
// per lane.  A lane sums the 27 contributions of a run of particles with the same nearest mesh
// point in registers and adds them once.  The adds go to an LDS box of mesh points, which is
// then added to the mesh with one global atomic per nonzero point.  The box is chosen per group
// of lanes: the whole wave's particles if the mesh points their clouds touch fit kAssignTile
// words; otherwise each half-wave's in a box of kAssignTile / 2 words, then each quarter's and
// each eighth's, taking for every group the largest one that fits.  A group of 8 << l lanes
// (level l) owns words [g, g + 1) * (kAssignTile / 8 << l) of the tile, g = lane / (8 << l),
// so the boxes of one wave never overlap.  An eighth that still does not fit (particles
// spread over a large region, or across the periodic seam) adds to the mesh directly.  Every
// sum is a fixed sequence of integer adds, so the mesh is the same on every run.
constexpr int kAssignThreads = 64;
constexpr int kAssignPer = 4;
constexpr int kAssignChunk = kAssignThreads * kAssignPer;
constexpr int kAssignTile = 4096;
constexpr int kAssignSlot = kAssignTile / 8;  // words owned by eight lanes

__global__ __launch_bounds__(kAssignThreads) void k_pm_assign(
    const double4 *__restrict__ ps, int64_t n, int N, double inv_h,
    const unsigned long long *__restrict__ mx, unsigned long long *__restrict__ mass)
{
    __shared__ unsigned long long tile[kAssignTile];
    const int lane = threadIdx.x;
    // neighbouring chunks on one XCD, so their mesh points share its L2
    const int64_t first = (int64_t)xcd_block(blockIdx.x, gridDim.x) * kAssignChunk +
                          (int64_t)lane * kAssignPer;
    int lo[3] = {0x7fffffff, 0x7fffffff, 0x7fffffff}, hi[3] = {-0x7fffffff, -0x7fffffff, -0x7fffffff};
#pragma unroll
    for (int k = 0; k < kAssignPer; ++k) {
        if (first + k < n) {
            const double4 p = ps[first + k];
            const int c[3] = {nearest(p.x, inv_h), nearest(p.y, inv_h), nearest(p.z, inv_h)};
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                lo[a] = min(lo[a], c[a]);
                hi[a] = max(hi[a], c[a]);
            }
        }
    }
    // Bounding boxes of the lane's groups of 8, 16, 32 and 64 lanes (one butterfly), and the
    // largest group whose box fits its share of the tile.  All lanes of a group see the same
    // boxes for it and for every larger group, so they agree on the level.
    int base = 0, ox = 0, oy = 0, oz = 0, ey = 1, ez = 1, cells = 0;
    bool local = false;
    {
#pragma unroll
        for (int d = 1; d < 8; d <<= 1)
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                lo[a] = min(lo[a], __shfl_xor(lo[a], d, 64));
                hi[a] = max(hi[a], __shfl_xor(hi[a], d, 64));
            }
        int glo[4][3], ghi[4][3];
#pragma unroll
        for (int l = 0; l < 4; ++l) {
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                glo[l][a] = lo[a];
                ghi[l][a] = hi[a];
            }
            if (l < 3) {
                const int d = 8 << l;
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    lo[a] = min(lo[a], __shfl_xor(lo[a], d, 64));
                    hi[a] = max(hi[a], __shfl_xor(hi[a], d, 64));
                }
            }
        }
#pragma unroll
        for (int l = 3; l >= 0; --l) {
            if (local) continue;
            const int cap = kAssignSlot << l;
            if (glo[l][0] > ghi[l][0]) {  // no particles in this group (ragged tail)
                local = true;
                base = (lane >> (3 + l)) * cap;
                cells = 0;
                continue;
            }
            const int ex = ghi[l][0] - glo[l][0] + 3, fy = ghi[l][1] - glo[l][1] + 3,
                      fz = ghi[l][2] - glo[l][2] + 3;
            if ((int64_t)ex * fy * fz <= cap) {
                local = true;
                base = (lane >> (3 + l)) * cap;
                cells = ex * fy * fz;
                ox = glo[l][0] - 1;
                oy = glo[l][1] - 1;
                oz = glo[l][2] - 1;
                ey = fy;
                ez = fz;
            }
        }
    }
    // Word t of slot q (words q * kAssignSlot ...) belongs to the box of lane 8 q's group: it is
    // used iff t - base < cells there (base and cells of a direct group are 0).
#pragma unroll 1
    for (int q = 0; q < 8; ++q) {
        const int qb = __shfl(base, 8 * q, 64), qc = __shfl(cells, 8 * q, 64);
#pragma unroll
        for (int j = 0; j < kAssignSlot / kAssignThreads; ++j) {
            const int t = q * kAssignSlot + j * kAssignThreads + lane;
            if (t - qb < qc) tile[t] = 0ull;
        }
    }
    __syncthreads();
    const double S = pm_scale(*mx, n);
    const int mask = N - 1;
    double acc[27];
#pragma unroll
    for (int j = 0; j < 27; ++j) acc[j] = 0.0;
    int cx = 0, cy = 0, cz = 0;
    bool open = false;
    auto add_run = [&]() {
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b)
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const unsigned long long v = __double2ull_rn(acc[(a * 3 + b) * 3 + c]);
                    if (local)
                        atomicAdd(&tile[base + ((cx - 1 + a - ox) * ey + (cy - 1 + b - oy)) * ez +
                                        (cz - 1 + c - oz)],
                                  v);
                    else
                        atomicAdd(&mass[((size_t)((cx - 1 + a) & mask) * N +
                                         ((cy - 1 + b) & mask)) * N + ((cz - 1 + c) & mask)],
                                  v);
                }
    };
#pragma unroll
    for (int k = 0; k < kAssignPer; ++k) {
        if (first + k < n) {
            const double4 p = ps[first + k];
            double wx[3], wy[3], wz[3];
            const int ix = tsc(p.x, inv_h, wx), iy = tsc(p.y, inv_h, wy), iz = tsc(p.z, inv_h, wz);
            if (open && (ix != cx || iy != cy || iz != cz)) {
                add_run();
#pragma unroll
                for (int j = 0; j < 27; ++j) acc[j] = 0.0;
            }
            cx = ix;
            cy = iy;
            cz = iz;
            open = true;
            const double ms = p.w * S;
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int b = 0; b < 3; ++b) {
                    const double wab = ms * wx[a] * wy[b];
#pragma unroll
                    for (int c = 0; c < 3; ++c) acc[(a * 3 + b) * 3 + c] += wab * wz[c];
                }
        }
    }
    if (open) add_run();
    __syncthreads();
#pragma unroll 1
    for (int q = 0; q < 8; ++q) {
        const int qb = __shfl(base, 8 * q, 64), qc = __shfl(cells, 8 * q, 64);
        const int qx = __shfl(ox, 8 * q, 64), qy = __shfl(oy, 8 * q, 64),
                  qz = __shfl(oz, 8 * q, 64), qey = __shfl(ey, 8 * q, 64),
                  qez = __shfl(ez, 8 * q, 64);
        for (int j = 0; j < kAssignSlot / kAssignThreads; ++j) {
            const int t = q * kAssignSlot + j * kAssignThreads + lane;
            const int u = t - qb;
            if (u >= qc) continue;
            const unsigned long long v = tile[t];
            if (!v) continue;
            const int lz = u % qez, ly = (u / qez) % qey, lx = u / (qez * qey);
            atomicAdd(&mass[((size_t)((qx + lx) & mask) * N + ((qy + ly) & mask)) * N +
                            ((qz + lz) & mask)],
                      v);
        }
    }
}

// ---------------------------------------------------------------- FFT on bundles of lines

struct Bundle {
    int N, logN, B, p, q0;
};

__device__ __forceinline__ Bundle bundle(int N, int logN, int B)
{
    Bundle u;
    u.N = N;
    u.logN = logN;
    u.B = B;
    const int per_row = N / B;
    u.p = blockIdx.x / per_row;
    u.q0 = (blockIdx.x % per_row) * B;
    return u;
}

// Global address of element e of line l of the bundle, for the transform along AXIS.
template <int AXIS>
__device__ __forceinline__ size_t elem_addr(const Bundle &u, int l, int e)
{
    const size_t N = u.N, NN = N * N;
    if (AXIS == 0) return (size_t)e * NN + (size_t)u.p * N + u.q0 + l;
    if (AXIS == 1) return (size_t)u.p * NN + (size_t)e * N + u.q0 + l;
    return (size_t)u.p * NN + (size_t)(u.q0 + l) * N + e;
}

// LDS slot of element e of line l: element-major along x and y (so a row of B lines is
// contiguous), line-major along z.
template <int AXIS>
__device__ __forceinline__ int slot(const Bundle &u, int l, int e)
{
    return AXIS == 2 ? l * u.N + e : e * u.B + l;
}

// The j-th of the loaded values, in the order that makes global reads contiguous.
template <int AXIS>
__device__ __forceinline__ void item(const Bundle &u, int j, int &l, int &e)
{
    if (AXIS == 2) {
        l = j >> u.logN;
        e = j & (u.N - 1);
    } else {
        e = j / u.B;
        l = j % u.B;
    }
}

// Butterfly b of a stage: its line and its index within the line.
template <int AXIS>
__device__ __forceinline__ void fly(const Bundle &u, int b, int &l, int &bb)
{
    if (AXIS == 2) {
        l = b >> (u.logN - 1);
        bb = b & ((u.N >> 1) - 1);
    } else {
        l = b % u.B;
        bb = b / u.B;
    }
}

// Decimation in time: input in bit-reversed order, output in natural order.  INV uses the
// conjugate twiddles (an unnormalised inverse transform).
template <int AXIS, int INV>
__device__ __forceinline__ void fft_dit(const Bundle &u, float2 *buf, const float2 *tw)
{
    const int tot = u.B * u.N;
    for (int s = 1; s <= u.logN; ++s) {
        const int half = 1 << (s - 1);
        for (int b = threadIdx.x; b < tot / 2; b += kFftThreads) {
            int l, bb;
            fly<AXIS>(u, b, l, bb);
            const int j = bb & (half - 1);
            const int k0 = ((bb >> (s - 1)) << s) + j, k1 = k0 + half;
            float2 w = tw[j << (u.logN - s)];
            if (INV) w.y = -w.y;
            const float2 x0 = buf[slot<AXIS>(u, l, k0)];
            const float2 t = cmul(w, buf[slot<AXIS>(u, l, k1)]);
            buf[slot<AXIS>(u, l, k0)] = cadd(x0, t);
            buf[slot<AXIS>(u, l, k1)] = csub(x0, t);
        }
        __syncthreads();
    }
}

// Decimation in frequency: input in natural order, output in bit-reversed order.
template <int AXIS, int INV>
__device__ __forceinline__ void fft_dif(const Bundle &u, float2 *buf, const float2 *tw)
{
    const int tot = u.B * u.N;
    for (int s = u.logN; s >= 1; --s) {
        const int half = 1 << (s - 1);
        for (int b = threadIdx.x; b < tot / 2; b += kFftThreads) {
            int l, bb;
            fly<AXIS>(u, b, l, bb);
            const int j = bb & (half - 1);
            const int k0 = ((bb >> (s - 1)) << s) + j, k1 = k0 + half;
            float2 w = tw[j << (u.logN - s)];
            if (INV) w.y = -w.y;
            const float2 x0 = buf[slot<AXIS>(u, l, k0)], x1 = buf[slot<AXIS>(u, l, k1)];
            buf[slot<AXIS>(u, l, k0)] = cadd(x0, x1);
            buf[slot<AXIS>(u, l, k1)] = cmul(csub(x0, x1), w);
        }
        __syncthreads();
    }
}

__device__ __forceinline__ int bitrev(int e, int logN) { return (int)(__brev((unsigned)e) >> (32 - logN)); }

__device__ __forceinline__ void load_twiddles(float2 *tw_s, const float2 *tw, int N)
{
    for (int k = threadIdx.x; k < N / 2; k += kFftThreads) tw_s[k] = tw[k];
}

// Transform along x or y (AXIS 0, 1) or z without the Green's function (not used), forward or
// inverse.  SRC: 0 complex mesh, 1 fixed-point masses (scaled by 1/S into the real part).
// DST: 0 complex mesh, 1 real part only (the potential).
template <int AXIS, int INV, int SRC, int DST>
__global__ __launch_bounds__(kFftThreads) void k_fft(float2 *__restrict__ a,
                                                     const unsigned long long *__restrict__ mass,
                                                     const unsigned long long *__restrict__ mx,
                                                     int64_t n_part, float *__restrict__ phi,
                                                     int N, int logN, int B,
                                                     const float2 *__restrict__ tw)
{
    __shared__ float2 buf[kFftElems];
    __shared__ float2 tw_s[kMaxTwiddles];
    const Bundle u = bundle(N, logN, B);
    load_twiddles(tw_s, tw, N);
    const int tot = B * N;
    const double inv_s = SRC ? 1.0 / pm_scale(*mx, n_part) : 1.0;
    for (int j = threadIdx.x; j < tot; j += kFftThreads) {
        int l, e;
        item<AXIS>(u, j, l, e);
        const size_t g = elem_addr<AXIS>(u, l, e);
        float2 v;
        if (SRC)
            v = make_float2((float)((double)mass[g] * inv_s), 0.0f);
        else
            v = a[g];
        buf[slot<AXIS>(u, l, bitrev(e, logN))] = v;
    }
    __syncthreads();
    fft_dit<AXIS, INV>(u, buf, tw_s);
    for (int j = threadIdx.x; j < tot; j += kFftThreads) {
        int l, e;
        item<AXIS>(u, j, l, e);
        const size_t g = elem_addr<AXIS>(u, l, e);
        if (DST)
            phi[g] = buf[slot<AXIS>(u, l, e)].x;
        else
            a[g] = buf[slot<AXIS>(u, l, e)];
    }
}

// z forward, times the Green's function, z inverse.  After the x and y forward passes the
// bundle's lines are at wavenumbers (kx, ky) = (p, q0 + l); after the DIF the value at
// position r of a line is at kz = bitrev(r).  green is the octant table, index
// (fx H + fy) H + fz with f = min(k, N - k), H = N/2 + 1.
__global__ __launch_bounds__(kFftThreads) void k_fft_z_green(float2 *__restrict__ a, int N,
                                                             int logN, int B,
                                                             const float2 *__restrict__ tw,
                                                             const float *__restrict__ green)
{
    __shared__ float2 buf[kFftElems];
    __shared__ float2 tw_s[kMaxTwiddles];
    const Bundle u = bundle(N, logN, B);
    load_twiddles(tw_s, tw, N);
    const int tot = B * N;
    for (int j = threadIdx.x; j < tot; j += kFftThreads) {
        int l, e;
        item<2>(u, j, l, e);
        buf[slot<2>(u, l, e)] = a[elem_addr<2>(u, l, e)];
    }
    __syncthreads();
    fft_dif<2, 0>(u, buf, tw_s);
    const int H = N / 2 + 1;
    const int fx = u.p <= N / 2 ? u.p : N - u.p;
    for (int j = threadIdx.x; j < tot; j += kFftThreads) {
        int l, r;
        item<2>(u, j, l, r);
        const int ky = u.q0 + l, kz = bitrev(r, logN);
        const int fy = ky <= N / 2 ? ky : N - ky, fz = kz <= N / 2 ? kz : N - kz;
        const float gk = green[((size_t)fx * H + fy) * H + fz];
        const float2 v = buf[slot<2>(u, l, r)];
        buf[slot<2>(u, l, r)] = make_float2(v.x * gk, v.y * gk);
    }
    __syncthreads();
    fft_dit<2, 1>(u, buf, tw_s);
    for (int j = threadIdx.x; j < tot; j += kFftThreads) {
        int l, e;
        item<2>(u, j, l, e);
        a[elem_addr<2>(u, l, e)] = buf[slot<2>(u, l, e)];
    }
}

// Fourier transform of the S2 cloud of radius eta at x = k eta (Hockney & Eastwood's shape):
// 12 (2 - 2 cos x - x sin x) / x^4, by its Taylor series where the closed form cancels.
__device__ __forceinline__ double s2_hat(double x)
{
    if (x < 0.2) {
        const double x2 = x * x;
        return 1.0 - x2 / 15.0 + x2 * x2 / 560.0 - x2 * x2 * x2 / 37800.0;
    }
    double sn, cs;
    sincos(x, &sn, &cs);
    const double x2 = x * x;
    return 12.0 * (2.0 - 2.0 * cs - x * sn) / (x2 * x2);
}

// Green's function octant table and twiddles.  G(k) = -4 pi S^(k eta)^2 / (k^2 W(k)^2 L^3):
// the long-range potential of a unit mass (the force between two S2 clouds of radius eta,
// whose complement is eq. 2) over the TSC window W = prod sinc^3(k_a h / 2) divided out for
// both the assignment and the interpolation, and 1/L^3 of the inverse transform; G(0) = 0.
// tw[k] = exp(-2 pi i k / N), k < N/2.
__global__ __launch_bounds__(256) void k_pm_green(int N, double L, double eta,
                                                  float *__restrict__ green,
                                                  float2 *__restrict__ tw)
{
    const int H = N / 2 + 1;
    const size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (t < (size_t)N / 2) {
        double sn, cs;
        sincospi(2.0 * (double)t / N, &sn, &cs);
        tw[t] = make_float2((float)cs, (float)-sn);
    }
    if (t >= (size_t)H * H * H) return;
    const int fz = (int)(t % H), fy = (int)((t / H) % H), fx = (int)(t / ((size_t)H * H));
    const double kf = 2.0 * M_PI / L, h = L / N;
    const int f[3] = {fx, fy, fz};
    double k2 = 0.0, W = 1.0;
    for (int a = 0; a < 3; ++a) {
        const double k = kf * f[a];
        k2 += k * k;
        const double x = 0.5 * k * h;
        const double sc = f[a] ? sin(x) / x : 1.0;
        W *= sc * sc * sc;
    }
    if (k2 == 0.0) {
        green[t] = 0.0f;
        return;
    }
    const double S = s2_hat(sqrt(k2) * eta);
    green[t] = (float)(-4.0 * M_PI * S * S / (k2 * W * W * L * L * L));
}

// F_a = -[(2/3)(phi(i+1) - phi(i-1)) - (1/12)(phi(i+2) - phi(i-2))] / h along each axis,
// stored as (Fx, Fy, Fz, 0) per mesh point so that interpolation reads one 16-byte word.
__global__ __launch_bounds__(256) void k_pm_fd(const float *__restrict__ phi, int N, int logN,
                                               float inv_h, float4 *__restrict__ f)
{
    const size_t t = xcd_block(blockIdx.x, gridDim.x) * (size_t)blockDim.x + threadIdx.x;
    const size_t NN = (size_t)N * N;
    if (t >= NN * N) return;
    const int m = N - 1;
    const int z = (int)(t & m), y = (int)((t >> logN) & m), x = (int)(t >> (2 * logN));
    const size_t rx = (size_t)y * N + z, ry = (size_t)x * NN + z, rz = (size_t)x * NN + (size_t)y * N;
    const float c1 = 2.0f / 3.0f, c2 = 1.0f / 12.0f;
    auto d = [&](float p1, float m1, float p2, float m2) {
        return -(c1 * (p1 - m1) - c2 * (p2 - m2)) * inv_h;
    };
    f[t] = make_float4(
        d(phi[(size_t)((x + 1) & m) * NN + rx], phi[(size_t)((x - 1) & m) * NN + rx],
          phi[(size_t)((x + 2) & m) * NN + rx], phi[(size_t)((x - 2) & m) * NN + rx]),
        d(phi[ry + (size_t)((y + 1) & m) * N], phi[ry + (size_t)((y - 1) & m) * N],
          phi[ry + (size_t)((y + 2) & m) * N], phi[ry + (size_t)((y - 2) & m) * N]),
        d(phi[rz + ((z + 1) & m)], phi[rz + ((z - 1) & m)], phi[rz + ((z + 2) & m)],
          phi[rz + ((z - 2) & m)]),
        0.0f);
}

// TSC interpolation of the mesh force to each particle, taken in key order, written to
// stage[idx[i]] = (ax, ay, az, 0), i.e. already in the caller's order.  Neighbouring threads
// hold neighbouring particles, so the 27-point gathers mostly hit the same cache lines; each
// thread writes one whole 16-byte record (k_pm_split then writes the three arrays
// contiguously).
__global__ __launch_bounds__(256) void k_pm_interp(const double4 *__restrict__ ps, int64_t n,
                                                   int N, double inv_h,
                                                   const float4 *__restrict__ f,
                                                   const uint32_t *__restrict__ idx,
                                                   float4 *__restrict__ stage)
{
    const int64_t i = xcd_block(blockIdx.x, gridDim.x) * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double4 p = ps[i];
    double wx[3], wy[3], wz[3];
    const int ix = tsc(p.x, inv_h, wx), iy = tsc(p.y, inv_h, wy), iz = tsc(p.z, inv_h, wz);
    const int mask = N - 1;
    float sx = 0.0f, sy = 0.0f, sz = 0.0f;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const size_t xa = (size_t)((ix - 1 + a) & mask) * N;
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            const size_t yb = (xa + ((iy - 1 + b) & mask)) * N;
            const double wab = wx[a] * wy[b];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const float w = (float)(wab * wz[c]);
                const float4 v = f[yb + ((iz - 1 + c) & mask)];
                sx += w * v.x;
                sy += w * v.y;
                sz += w * v.z;
            }
        }
    }
    stage[idx[i]] = make_float4(sx, sy, sz, 0.0f);
}

// The caller's order o: ax[o], ay[o], az[o] = stage[o] (written, or added to with ACC).
template <typename T, int ACC>
__global__ __launch_bounds__(256) void k_pm_split(const float4 *__restrict__ stage, int64_t n,
                                               T *__restrict__ ax, T *__restrict__ ay,
                                               T *__restrict__ az)
{
    const int64_t o = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (o >= n) return;
    const float4 v = stage[o];
    if (ACC) {
        ax[o] += (T)v.x;
        ay[o] += (T)v.y;
        az[o] += (T)v.z;
    } else {
        ax[o] = (T)v.x;
        ay[o] = (T)v.y;
        az[o] = (T)v.z;
    }
}

} // namespace

int pm_bundle_lines(int N) { return N >= 256 ? kFftElems / N : (N < 16 ? N : 16); }

void launch_pm_green(int N, double L, double eta, float *green, float2 *tw, hipStream_t s)
{
    const size_t H = N / 2 + 1;
    const size_t work = H * H * H > (size_t)N / 2 ? H * H * H : (size_t)N / 2;
    k_pm_green<<<(unsigned)((work + 255) / 256), 256, 0, s>>>(N, L, eta, green, tw);
}

void launch_pm_assign(const double4 *ps, int64_t n, int N, double L, unsigned long long *mx,
                      unsigned long long *mass, hipStream_t s)
{
    fill_u64((uint64_t *)mass, (size_t)N * N * N, 0ull, s);
    if (!n) return;
    k_pm_assign<<<(unsigned)((n + kAssignChunk - 1) / kAssignChunk), kAssignThreads, 0, s>>>(
        ps, n, N, N / L, mx, mass);
}

void launch_pm_potential(const unsigned long long *mass, const unsigned long long *mx,
                         int64_t n, int N, float2 *grid, float *phi, const float *green,
                         const float2 *tw, hipStream_t s)
{
    const int logN = __builtin_ctz((unsigned)N);
    const int B = pm_bundle_lines(N);
    const unsigned blocks = (unsigned)((size_t)N * N / B);
    k_fft<0, 0, 1, 0><<<blocks, kFftThreads, 0, s>>>(grid, mass, mx, n, nullptr, N, logN, B, tw);
    k_fft<1, 0, 0, 0><<<blocks, kFftThreads, 0, s>>>(grid, nullptr, nullptr, n, nullptr, N, logN,
                                                     B, tw);
    k_fft_z_green<<<blocks, kFftThreads, 0, s>>>(grid, N, logN, B, tw, green);
    k_fft<1, 1, 0, 0><<<blocks, kFftThreads, 0, s>>>(grid, nullptr, nullptr, n, nullptr, N, logN,
                                                     B, tw);
    k_fft<0, 1, 0, 1><<<blocks, kFftThreads, 0, s>>>(grid, nullptr, nullptr, n, phi, N, logN, B,
                                                     tw);
}

void launch_pm_force(const float *phi, int N, double L, float4 *f, hipStream_t s)
{
    const size_t pts = (size_t)N * N * N;
    k_pm_fd<<<(unsigned)((pts + 255) / 256), 256, 0, s>>>(phi, N, __builtin_ctz((unsigned)N),
                                                          (float)(N / L), f);
}

void launch_pm_interp(const double4 *ps, int64_t n, int N, double L, const float4 *f,
                      const uint32_t *idx, float4 *stage, hipStream_t s)
{
    if (!n) return;
    k_pm_interp<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(ps, n, N, N / L, f, idx, stage);
}

void launch_pm_split(const float4 *stage, int64_t n, void *ax, void *ay, void *az,
                     int out_fp64, int accumulate, hipStream_t s)
{
    if (!n) return;
    const unsigned b = (unsigned)((n + 255) / 256);
    if (out_fp64) {
        if (accumulate)
            k_pm_split<double, 1><<<b, 256, 0, s>>>(stage, n, (double *)ax, (double *)ay,
                                                (double *)az);
        else
            k_pm_split<double, 0><<<b, 256, 0, s>>>(stage, n, (double *)ax, (double *)ay,
                                                (double *)az);
    } else {
        if (accumulate)
            k_pm_split<float, 1><<<b, 256, 0, s>>>(stage, n, (float *)ax, (float *)ay, (float *)az);
        else
            k_pm_split<float, 0><<<b, 256, 0, s>>>(stage, n, (float *)ax, (float *)ay, (float *)az);
    }
}

} // namespace tpm
