// Particle-mesh (PM) long-range force on an N^3 periodic mesh (Section 2.2 step 1): TSC
// mass assignment, the potential by FFT with the Green's function of the long-range part of
// the split (the complement of eq. 2), a fourth-order difference for the mesh force and TSC
// interpolation back to the particles.
//
// Mesh layout: point (x, y, z) at (x N + y) N + z, z contiguous; N a power of two.
//  * assignment by owner cells: the mesh is cut into cells of 8^3 points (tree cells, so a
//    cell's particles are contiguous in key order); a workgroup sums a chunk of one cell's
//    particles into the cell's 11^3 box in LDS and stores the box to its own slot, then one
//    workgroup per cell adds, for each of its points, the slot words that cover it.  Masses
//    are 64-bit fixed point and every sum is a fixed set of integer adds, so the mesh is the
//    same on every run; there are no global atomics;
//  * FFT: complex, radix 2, one workgroup per bundle of B lines of one axis held in LDS
//    (B N = 4096 values, B <= 16).  Bundles along x and y are B neighbouring lines in z, so a
//    load of one element row is B contiguous values; bundles along z are B contiguous rows.
//    The passes are: x forward (reading the fixed-point masses), y forward, z forward +
//    Green's function + z inverse in one kernel (a DIF forward leaves bit-reversed order, which
//    is what the DIT inverse reads), y inverse, x inverse (writing the real potential);
//  * mesh force: fourth-order central differences of the potential, one float4 per point;
//  * interpolation: over the assignment's chunks, the cell's 11^3 box of force words read
//    into LDS once, each particle's 27 words from there; the 16-byte result goes to the
//    particle's slot in the caller's order through the sort permutation (a scattered write);
//    k_pm_split then writes the three output arrays contiguously.
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

// Mass assignment, owner by owner.  The mesh is cut into cells of kCellPts^3 points, which
// are the tree cells of level l_c = log2(N / kCellPts): a particle's cell c (per axis) is its
// key's prefix, and its nearest mesh point i0 = floor(x N / L + 1/2) lies in [8c, 8c + 8] (the
// key's product x 2^21 / L and x N / L differ from the exact values by a relative 2^-52 at
// most, far below the half point of margin; at x -> L the key is clamped and i0 = N, still in
// range).  So the particles of a cell, contiguous in key order, touch only the kBox^3 points
// [8c - 1, 8c + 9] of the cell's box.  One workgroup sums a chunk of a cell's particles into
// its box in LDS and writes the box to the chunk's own slot with plain stores; then each mesh
// point sums the slot words that cover it (one or two cells per axis, every chunk of each) and
// writes its mesh word.  No global atomics, and every sum is a fixed set of integer adds, so
// the mesh is the same on every run.  A thread sums the 27 contributions of a run of its
// particles with the same nearest point in registers (fixed point, rounded once per run and
// point).
constexpr int kCellPts = 8;
constexpr int kBox = kCellPts + 3;             // 11 points per axis
constexpr int kBoxWords = kBox * kBox * kBox;  // 1331
constexpr int kCellChunk = 4096;               // particles per workgroup at most
constexpr int kAssignThreads = 256;

__device__ __forceinline__ uint32_t spread3_10(uint32_t v) // 10 bits -> every third bit
{
    v &= 0x3ffu;
    v = (v | (v << 16)) & 0x030000ffu;
    v = (v | (v << 8)) & 0x0300f00fu;
    v = (v | (v << 4)) & 0x030c30c3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}
__device__ __forceinline__ uint32_t compact3_10(uint32_t v)
{
    v &= 0x09249249u;
    v = (v | (v >> 2)) & 0x030c30c3u;
    v = (v | (v >> 4)) & 0x0300f00fu;
    v = (v | (v >> 8)) & 0x030000ffu;
    v = (v | (v >> 16)) & 0x3ffu;
    return v;
}
// The Morton index of cell (cx, cy, cz), in the keys' bit order (x above y above z).
__device__ __forceinline__ uint32_t cell_index(uint32_t cx, uint32_t cy, uint32_t cz)
{
    return (spread3_10(cx) << 2) | (spread3_10(cy) << 1) | spread3_10(cz);
}

// cell_start[m] = the first particle (key order) of Morton cell m, m = 0 .. ncells; the
// cell of a key is key >> sh.
__global__ __launch_bounds__(256) void k_pm_cells(const uint64_t *__restrict__ key, int64_t n,
                                                  int sh, uint32_t ncells,
                                                  uint32_t *__restrict__ cell_start)
{
    const uint32_t m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m > ncells) return;
    int64_t lo = 0, hi = n; // first i with key[i] >> sh >= m
    while (lo < hi) {
        const int64_t mid = lo + ((hi - lo) >> 1);
        if ((key[mid] >> sh) < (uint64_t)m)
            lo = mid + 1;
        else
            hi = mid;
    }
    cell_start[m] = (uint32_t)lo;
}

// items[m] = chunks of cell m (exclusive prefix taken afterwards).
__global__ __launch_bounds__(256) void k_pm_cell_items(const uint32_t *__restrict__ cell_start,
                                                       uint32_t ncells,
                                                       uint32_t *__restrict__ items)
{
    const uint32_t m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= ncells) return;
    const uint32_t c = cell_start[m + 1] - cell_start[m];
    items[m] = (c + kCellChunk - 1) / kCellChunk;
}

// The cell whose chunks include chunk `item`: the last m with item_start[m] <= item.
__device__ __forceinline__ uint32_t item_cell(const uint32_t *__restrict__ item_start,
                                              uint32_t ncells, uint32_t item)
{
    uint32_t lo = 0, hi = ncells;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (item_start[mid] <= item)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

// One workgroup per chunk (grid: an upper bound on the chunks; the rest leave).
__global__ __launch_bounds__(kAssignThreads) void k_pm_assign(
    const double4 *__restrict__ ps, int64_t n, int N, double inv_h,
    const unsigned long long *__restrict__ mx, const uint32_t *__restrict__ cell_start,
    const uint32_t *__restrict__ item_start, uint32_t ncells,
    unsigned long long *__restrict__ slots)
{
    __shared__ unsigned long long box[kBoxWords];
    const uint32_t item = blockIdx.x;
    if (item >= item_start[ncells]) return; // the same for the whole workgroup
    const uint32_t m = item_cell(item_start, ncells, item);
    const uint32_t first = cell_start[m] + (item - item_start[m]) * (uint32_t)kCellChunk;
    const uint32_t end = min(cell_start[m + 1], first + (uint32_t)kCellChunk);
    const int ox = 8 * (int)compact3_10(m >> 2) - 1, oy = 8 * (int)compact3_10(m >> 1) - 1,
              oz = 8 * (int)compact3_10(m) - 1;
    for (int t = threadIdx.x; t < kBoxWords; t += kAssignThreads) box[t] = 0ull;
    __syncthreads();
    const double S = pm_scale(*mx, n);
    const uint32_t per = (end - first + kAssignThreads - 1) / kAssignThreads;
    const uint32_t i0 = first + threadIdx.x * per, i1 = min(end, i0 + per);
    double acc[27];
#pragma unroll
    for (int j = 0; j < 27; ++j) acc[j] = 0.0;
    int cx = 0, cy = 0, cz = 0;
    bool open = false;
    auto add_run = [&]() {
        const int bx = cx - 1 - ox, by = cy - 1 - oy, bz = cz - 1 - oz; // in [0, 8]
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b)
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const unsigned long long v = __double2ull_rn(acc[(a * 3 + b) * 3 + c]);
                    if (v) atomicAdd(&box[((bx + a) * kBox + (by + b)) * kBox + (bz + c)], v);
                }
    };
    for (uint32_t i = i0; i < i1; ++i) {
        const double4 p = ps[i];
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
    if (open) add_run();
    __syncthreads();
    unsigned long long *dst = slots + (size_t)item * kBoxWords;
    for (int t = threadIdx.x; t < kBoxWords; t += kAssignThreads) dst[t] = box[t];
}

// One workgroup per cell, one thread per mesh point of the cell: the sum of the slot words of
// every chunk of every cell whose box covers the point (its own cell, and the neighbour on
// the low side for the cell's first two planes, on the high side for its last plane, per
// axis).  The 27 neighbours' chunk ranges are read into LDS once.
__global__ __launch_bounds__(kCellPts * kCellPts * kCellPts) void k_pm_gather(
    int N, const uint32_t *__restrict__ item_start, const unsigned long long *__restrict__ slots,
    unsigned long long *__restrict__ mass)
{
    __shared__ uint32_t rng[27][2];
    const int ncell = N / kCellPts, cm = ncell - 1;
    // each XCD takes a contiguous slab of cells, whose neighbours' slots its L2 then shares
    const int cell = (int)xcd_block(blockIdx.x, gridDim.x);
    const int cx = cell / (ncell * ncell), cy = (cell / ncell) % ncell, cz = cell % ncell;
    const int t = threadIdx.x;
    if (t < 27) {
        const int dx = t / 9 - 1, dy = (t / 3) % 3 - 1, dz = t % 3 - 1;
        const uint32_t m = cell_index((uint32_t)((cx + dx) & cm), (uint32_t)((cy + dy) & cm),
                                      (uint32_t)((cz + dz) & cm));
        rng[t][0] = item_start[m];
        rng[t][1] = item_start[m + 1];
    }
    __syncthreads();
    const int x0 = t >> 6, y0 = (t >> 3) & 7, z0 = t & 7; // point within the cell
    unsigned long long sum = 0ull;
    for (int dx = -1; dx <= 1; ++dx) {
        const int lx = x0 - 8 * dx + 1; // the point in the box of neighbour dx
        if (lx < 0 || lx >= kBox) continue;
        for (int dy = -1; dy <= 1; ++dy) {
            const int ly = y0 - 8 * dy + 1;
            if (ly < 0 || ly >= kBox) continue;
            for (int dz = -1; dz <= 1; ++dz) {
                const int lz = z0 - 8 * dz + 1;
                if (lz < 0 || lz >= kBox) continue;
                const int k = ((dx + 1) * 3 + (dy + 1)) * 3 + (dz + 1);
                const int w = (lx * kBox + ly) * kBox + lz;
                for (uint32_t it = rng[k][0]; it < rng[k][1]; ++it)
                    sum += slots[(size_t)it * kBoxWords + w];
            }
        }
    }
    mass[((size_t)(8 * cx + x0) * N + (size_t)(8 * cy + y0)) * N + (size_t)(8 * cz + z0)] = sum;
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

// TSC interpolation of the mesh force to each particle, written to stage[idx[i]] =
// (ax, ay, az, 0), i.e. already in the caller's order (k_pm_split then writes the three arrays
// contiguously).  One workgroup per chunk of a cell's particles (the chunks of the
// assignment): the kBox^3 force words around the cell, [8c - 1, 8c + 9] per axis, are read
// into LDS once, and each particle's 27 words come from there.  The weights and the order of
// the sums are those of a plain per-particle gather.
__global__ __launch_bounds__(kAssignThreads) void k_pm_interp(
    const double4 *__restrict__ ps, int N, double inv_h, const float4 *__restrict__ f,
    const uint32_t *__restrict__ idx, float4 *__restrict__ stage,
    const uint32_t *__restrict__ cell_start, const uint32_t *__restrict__ item_start,
    uint32_t ncells)
{
    __shared__ float4 box[kBoxWords];
    // each XCD takes a contiguous run of chunks (cells in Morton order): the chunks of one
    // cell and its neighbours then read their boxes through one L2
    const uint32_t item = xcd_block(blockIdx.x, gridDim.x);
    if (item >= item_start[ncells]) return; // the same for the whole workgroup
    const uint32_t m = item_cell(item_start, ncells, item);
    const uint32_t first = cell_start[m] + (item - item_start[m]) * (uint32_t)kCellChunk;
    const uint32_t end = min(cell_start[m + 1], first + (uint32_t)kCellChunk);
    const int ox = 8 * (int)compact3_10(m >> 2) - 1, oy = 8 * (int)compact3_10(m >> 1) - 1,
              oz = 8 * (int)compact3_10(m) - 1;
    const int mask = N - 1;
    for (int t = threadIdx.x; t < kBoxWords; t += kAssignThreads) {
        const int bx = t / (kBox * kBox), by = (t / kBox) % kBox, bz = t % kBox;
        box[t] = f[((size_t)((ox + bx) & mask) * N + ((oy + by) & mask)) * N + ((oz + bz) & mask)];
    }
    __syncthreads();
    for (uint32_t i = first + threadIdx.x; i < end; i += kAssignThreads) {
        const double4 p = ps[i];
        double wx[3], wy[3], wz[3];
        const int ix = tsc(p.x, inv_h, wx), iy = tsc(p.y, inv_h, wy), iz = tsc(p.z, inv_h, wz);
        const int bx = ix - 1 - ox, by = iy - 1 - oy, bz = iz - 1 - oz; // in [0, 8]
        float sx = 0.0f, sy = 0.0f, sz = 0.0f;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                const float4 *row = box + ((bx + a) * kBox + (by + b)) * kBox + bz;
                const double wab = wx[a] * wy[b];
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const float w = (float)(wab * wz[c]);
                    const float4 v = row[c];
                    sx += w * v.x;
                    sy += w * v.y;
                    sz += w * v.z;
                }
            }
        }
        stage[idx[i]] = make_float4(sx, sy, sz, 0.0f);
    }
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

size_t pm_assign_cells(int N) { const size_t c = (size_t)N / kCellPts; return c * c * c; }
size_t pm_assign_items_max(int N, int64_t n)
{
    return pm_assign_cells(N) + (size_t)((n + kCellChunk - 1) / kCellChunk);
}
size_t pm_assign_slot_words() { return kBoxWords; }

void launch_pm_assign(const double4 *ps, const uint64_t *key, int64_t n, int N, double L,
                      const unsigned long long *mx, uint32_t *cell_start, uint32_t *item_start,
                      uint32_t *scan_tmp, unsigned long long *slots, unsigned long long *mass,
                      hipStream_t s)
{
    const uint32_t ncells = (uint32_t)pm_assign_cells(N);
    const int lc = __builtin_ctz((unsigned)(N / kCellPts)); // tree level of the cells
    const int sh = 3 * (21 - lc);
    k_pm_cells<<<(ncells + 1 + 255) / 256, 256, 0, s>>>(key, n, sh, ncells, cell_start);
    k_pm_cell_items<<<(ncells + 255) / 256, 256, 0, s>>>(cell_start, ncells, item_start);
    scan_u32(item_start, ncells, item_start + ncells, scan_tmp, s); // exclusive; the total last
    const size_t items = pm_assign_items_max(N, n);
    if (n)
        k_pm_assign<<<(unsigned)items, kAssignThreads, 0, s>>>(ps, n, N, N / L, mx, cell_start,
                                                               item_start, ncells, slots);
    k_pm_gather<<<ncells, kCellPts * kCellPts * kCellPts, 0, s>>>(N, item_start, slots, mass);
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
                      const uint32_t *idx, float4 *stage, const uint32_t *cell_start,
                      const uint32_t *item_start, hipStream_t s)
{
    if (!n) return;
    const uint32_t ncells = (uint32_t)pm_assign_cells(N);
    k_pm_interp<<<(unsigned)pm_assign_items_max(N, n), kAssignThreads, 0, s>>>(
        ps, N, N / L, f, idx, stage, cell_start, item_start, ncells);
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
