// Short-range pair force over the interaction lists (Section 2.1 eq. 1 with the cutoff
// g_P3M of eq. 2 and Plummer softening of Section 2.4):
//
//   a_i += m_j d g(|d| / eta) / (|d|^2 + eps^2)^(3/2),   d = x_j - x_i.
//
// One 64-lane wavefront per group: the group's i-particles sit in registers and its list is
// streamed through LDS in tiles; lanes of one stream read the same tile entry (an LDS
// broadcast) and accumulate in registers.
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


// First branch of eq. (2) alone, for separations known to be below eta (R < 1).
__device__ __forceinline__ double g_in_f64(double R)
{
    double R2 = R * R;
    double p = fma(0.15, R, -12.0 / 35.0);
    p = fma(p, R, -0.5);
    p = fma(p, R, 1.6);
    p = fma(p, R2, -1.6);
    return fma(p, R2 * R, 1.0);
}

__device__ __forceinline__ double g_p3m_f64(double R)
{
    double g1 = g_in_f64(R);
    double u = fmax(2.0 - R, 0.0);
    double u2 = u * u;
    double u5 = u2 * u2 * u;
    double c = fma(fma(fma(0.05, R, 22.0 / 140.0), R, 10.0 / 140.0), R, 4.0 / 140.0);
    return R < 1.0 ? g1 : u5 * c;
}

// Second branch of eq. (2) alone, for separations known to be at least eta (R >= 1).
__device__ __forceinline__ double g_far_f64(double R)
{
    double u = fmax(2.0 - R, 0.0);
    double u2 = u * u;
    double u5 = u2 * u2 * u;
    double c = fma(fma(fma(0.05, R, 22.0 / 140.0), R, 10.0 / 140.0), R, 4.0 / 140.0);
    return u5 * c;
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

// FP32 path.  Lengths are in units of eta (the cutoff scale), so R = |d| and R^2 = |d|^2
// come for free; the sum is multiplied by 1/eta^2 once per particle:
//   a_i = (1/eta^2) sum_j m_j d'_ij g(|d'_ij|) / (|d'_ij|^2 + (eps/eta)^2)^(3/2).
//
// One tile takes up to kTileF32 list entries.  Each lane examines kTileF32 / 64 of them and
// drops those whose source is at least r_cut from the group's bounding box: every pair they
// would form is at least r_cut apart and adds exactly zero (g = 0 for R >= 2).  Survivors at
// least eta from the box ("far": every pair has R >= 1, so only the second branch of g
// applies) are kept apart from the others ("near").  Both kinds are compacted in list order
// and stored by stream: near survivor e goes to stream e % J, slot e / J, counting up from
// the start of the stream's run; far survivor e to stream e % J, slot e / J counting down
// from its end.  Slots past the last survivor of a stream, in either part, are zero-mass
// padding (they add exactly 0).
constexpr int kTileF32 = 256;

struct GroupFrame {
    double xg0, xg1, xg2;   // x_g, origin of the relative coordinates
    double cg0, cg1, cg2;   // bbox centre
    double hg0, hg1, hg2;   // bbox half size
    double L, rc2, eta2, inv_eta;
};

struct TileCounts {
    int near, far;
};

// Slots per stream of a tile: n_near + n_far <= kTileF32 survivors need at most
// kTileF32 / J + 1 rows once both parts are padded to a multiple of J.
__device__ __forceinline__ int tile_rows(int J) { return kTileF32 / J + 1; }

constexpr int kTileRounds = kTileF32 / 64;

// The list entries of the tile starting at jb (jb < Lg), one per lane and round.  Slots past
// the list's end read its last entry and are dropped by load_tile_f32.  The caller issues
// these reads one tile ahead, so they are in flight while the previous tile is evaluated.
__device__ __forceinline__ void fetch_entries(const uint32_t *__restrict__ list, uint64_t jb,
                                              uint64_t Lg, uint32_t *ent)
{
    const int lane = threadIdx.x;
#pragma unroll
    for (int r = 0; r < kTileRounds; ++r) {
        const uint64_t j = jb + (uint64_t)(r * 64 + lane);
        ent[r] = list[j < Lg ? j : Lg - 1];
    }
}

__device__ __forceinline__ TileCounts load_tile_f32(float4 *tile, const uint32_t *ent,
                                                    uint64_t jb, uint64_t Lg, int J, int rows,
                                                    NodeArrays nd, const GroupFrame &F)
{
    constexpr int kR = kTileRounds;
    const int lane = threadIdx.x;
    const uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;
    int n_near = 0, n_far = 0;
    // All source reads are issued before any is used, with no branch between them, so a tile
    // waits for one memory latency rather than one per round.
    double4 srcs[kR];
#pragma unroll
    for (int r = 0; r < kR; ++r) {
        const double4 *base = (ent[r] & kCellTag) ? nd.nsrc : nd.psrc;
        srcs[r] = base[ent[r] & ~kCellTag];
    }
#pragma unroll
    for (int r = 0; r < kR; ++r) {
        const uint64_t j = jb + (uint64_t)(r * 64 + lane);
        bool keep = false, far = false;
        float4 v;
        if (j < Lg) {
            const double4 src = srcs[r];
            const double sx = src.x, sy = src.y, sz = src.z, sm = src.w;
            double w0 = fabs(wrapd(sx - F.cg0, F.L)) - F.hg0;
            double w1 = fabs(wrapd(sy - F.cg1, F.L)) - F.hg1;
            double w2 = fabs(wrapd(sz - F.cg2, F.L)) - F.hg2;
            w0 = w0 > 0.0 ? w0 : 0.0;
            w1 = w1 > 0.0 ? w1 : 0.0;
            w2 = w2 > 0.0 ? w2 : 0.0;
            const double gap2 = w0 * w0 + w1 * w1 + w2 * w2;
            keep = gap2 < F.rc2;
            far = gap2 >= F.eta2;
            v = make_float4((float)(wrapd(sx - F.xg0, F.L) * F.inv_eta),
                            (float)(wrapd(sy - F.xg1, F.L) * F.inv_eta),
                            (float)(wrapd(sz - F.xg2, F.L) * F.inv_eta), (float)sm);
        }
        const uint64_t mn = __ballot(keep && !far);
        const uint64_t mf = __ballot(keep && far);
        if (keep) {
            if (far) {
                const int e = n_far + (int)__popcll(mf & lt);
                tile[(e % J) * rows + rows - 1 - e / J] = v;
            } else {
                const int e = n_near + (int)__popcll(mn & lt);
                tile[(e % J) * rows + e / J] = v;
            }
        }
        n_near += (int)__popcll(mn);
        n_far += (int)__popcll(mf);
    }
    // zero the padding slots of the last row of each part
    const float4 zero = make_float4(0.f, 0.f, 0.f, 0.f);
    const int en = n_near + lane;
    if (lane < J && en < (n_near + J - 1) / J * J) tile[(en % J) * rows + en / J] = zero;
    const int ef = n_far + lane - 32;
    if (lane >= 32 && lane < 32 + J && ef < (n_far + J - 1) / J * J)
        tile[(ef % J) * rows + rows - 1 - ef / J] = zero;
    TileCounts c;
    c.near = __builtin_amdgcn_readfirstlane(n_near);
    c.far = __builtin_amdgcn_readfirstlane(n_far);
    return c;
}

// Lane layout of a group of n_g particles on one wave: J streams of S = 64 / J lanes, each
// lane holding K = ceil(n_g / S) i-particles, each stream taking every J-th source.  Among
// J in {1, 2, 4, 8} with K <= 8 the layout with the fewest lane slots S * K is taken (the
// smallest J on ties), so few lanes idle: a group of 40 runs as 8 streams of 8 lanes with 5
// particles each (40 slots) rather than one stream of 64 lanes (64 slots).  Groups above 512
// run in chunks of 512 with J = 1, K = 8.
__host__ __device__ __forceinline__ void force_layout(uint32_t n_g, int &J, int &K)
{
    J = 1;
    K = 8;
    if (n_g > 512) return;
    uint32_t best = ~0u;
    for (int j = 1; j <= 8; j *= 2) {
        const uint32_t s = 64u / (uint32_t)j;
        uint32_t k = (n_g + s - 1) / s;
        k = k < 1 ? 1 : k;
        if (k <= 8 && s * k < best) {
            best = s * k;
            J = j;
            K = (int)k;
        }
    }
}

// Second branch of g (R >= 1, zero from R = 2 on) with u = clamp(1 - R/2, 0, 1), which is
// (2 - R)/2 exactly on [1, 2]:  (2 - R)^5 (7R^3 + 22R^2 + 10R + 4) / 140
//   = u^5 (1.6 R^3 + (704/140) R^2 + (320/140) R + 128/140).
// The factor 32 moved into the coefficients is a power of two, so the value is the same as
// with (2 - R) itself; the clamp is a modifier of the fma, not an instruction of its own.
__device__ __forceinline__ float g_far_f32(float R)
{
    const float u = fminf(fmaxf(fmaf(R, -0.5f, 1.0f), 0.0f), 1.0f);
    const float u2 = u * u;
    const float u5 = u2 * u2 * u;
    const float c =
        fmaf(fmaf(fmaf(1.6f, R, 704.0f / 140.0f), R, 320.0f / 140.0f), R, 128.0f / 140.0f);
    return u5 * c;
}

// g(R) of eq. (2) rearranged without cancellation; R2 = R * R is passed in.
__device__ __forceinline__ float g_p3m_f32s(float R, float R2)
{
    float p = fmaf(0.15f, R, -12.0f / 35.0f);
    p = fmaf(p, R, -0.5f);
    p = fmaf(p, R, 1.6f);
    p = fmaf(p, R2, -1.6f);
    const float g1 = fmaf(p, R2 * R, 1.0f);
    return R < 1.0f ? g1 : g_far_f32(R);
}

template <bool FAR>
__device__ __forceinline__ void pair_f32(const float4 s, float xi, float yi, float zi,
                                         float eps2, float &tx, float &ty, float &tz)
{
    const float dx = s.x - xi, dy = s.y - yi, dz = s.z - zi;
    const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
    const float rinv = __builtin_amdgcn_rsqf(r2 + eps2);
    const float rinv3 = rinv * rinv * rinv;
    const float R = __builtin_amdgcn_sqrtf(r2);
    const float g = FAR ? g_far_f32(R) : g_p3m_f32s(R, r2);
    const float fm = s.w * g * rinv3;
    tx = fmaf(fm, dx, tx);
    ty = fmaf(fm, dy, ty);
    tz = fmaf(fm, dz, tz);
}

// steps rows of a stream's tile run, starting at ts, against the lane's K i-particles.
template <int K, bool FAR>
__device__ __forceinline__ void tile_pass(const float4 *ts, int steps, const float *xi,
                                          const float *yi, const float *zi, float eps2,
                                          float *tx, float *ty, float *tz)
{
    int t = 0;
    if (K < 4) { // two rows per iteration; larger K has enough independent pairs per row
        for (; t + 2 <= steps; t += 2) {
            const float4 s0 = ts[t], s1 = ts[t + 1];
#pragma unroll
            for (int k = 0; k < K; ++k) {
                pair_f32<FAR>(s0, xi[k], yi[k], zi[k], eps2, tx[k], ty[k], tz[k]);
                pair_f32<FAR>(s1, xi[k], yi[k], zi[k], eps2, tx[k], ty[k], tz[k]);
            }
        }
    } else {
        for (; t + 1 < steps; ++t) {
            const float4 s0 = ts[t];
#pragma unroll
            for (int k = 0; k < K; ++k)
                pair_f32<FAR>(s0, xi[k], yi[k], zi[k], eps2, tx[k], ty[k], tz[k]);
        }
    }
    if (t < steps) {
        const float4 s0 = ts[t];
#pragma unroll
        for (int k = 0; k < K; ++k)
            pair_f32<FAR>(s0, xi[k], yi[k], zi[k], eps2, tx[k], ty[k], tz[k]);
    }
}

// Whether the next tile's list entries are read while the current tile is evaluated: only
// where the four extra registers do not push the class past its register budget (K = 5 and
// K = 7 sit at theirs).
__host__ __device__ constexpr bool force_prefetch(int K) { return K <= 4 || K == 6 || K == 8; }

// One group on one wave in the layout of force_layout (K i-particles per lane, J streams,
// each stream taking every J-th surviving source); the J partial sums are added at the end
// in stream order.
template <int K, int OUT64>
__device__ __forceinline__ void force_group_f32(float4 *tile, double *red, NodeArrays nd,
                                                uint32_t n_g, uint32_t f, const uint32_t *list,
                                                uint64_t Lg, const double4 *__restrict__ ps,
                                                const uint32_t *__restrict__ pidx,
                                                const GroupFrame &F, float eps2, double scale,
                                                void *ax, void *ay, void *az, uint32_t *kept_out)
{
    const int lane = threadIdx.x;
    int J, Kl;
    force_layout(n_g, J, Kl);
    (void)Kl;  // equals K: the group was classified with the same layout
    const int S = 64 / J;
    const int lgJ = J == 1 ? 0 : J == 2 ? 1 : J == 4 ? 2 : 3;
    const int slot = lane % S, stream = lane / S;
    const int rows = tile_rows(J);
    uint32_t kept_total = 0;
    for (uint32_t ib = 0; ib < n_g; ib += (uint32_t)(S * K)) {
        float xi[K], yi[K], zi[K], hx[K], hy[K], hz[K], lx[K], ly[K], lz[K];
        kept_total = 0;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const uint32_t i = ib + slot + S * k;
            xi[k] = yi[k] = zi[k] = 0.f;
            if (i < n_g) {
                const double4 r = ps[f + i];
                xi[k] = (float)((r.x - F.xg0) * F.inv_eta);
                yi[k] = (float)((r.y - F.xg1) * F.inv_eta);
                zi[k] = (float)((r.z - F.xg2) * F.inv_eta);
            }
            hx[k] = hy[k] = hz[k] = lx[k] = ly[k] = lz[k] = 0.f;
        }
        uint32_t ent[kTileRounds];
        if (force_prefetch(K) && Lg) fetch_entries(list, 0, Lg, ent);
        for (uint64_t jb = 0; jb < Lg; jb += kTileF32) {
            if (!force_prefetch(K)) fetch_entries(list, jb, Lg, ent);
            const TileCounts nt = load_tile_f32(tile, ent, jb, Lg, J, rows, nd, F);
            kept_total += (uint32_t)(nt.near + nt.far);
            __syncthreads();
            if (force_prefetch(K) && jb + kTileF32 < Lg)
                fetch_entries(list, jb + kTileF32, Lg, ent);
            // J is a power of two; the row counts are the same on every lane
            const int sn = (nt.near + J - 1) >> lgJ, sf = (nt.far + J - 1) >> lgJ;
            const float4 *ts = tile + stream * rows;
            float tx[K], ty[K], tz[K];
#pragma unroll
            for (int k = 0; k < K; ++k) tx[k] = ty[k] = tz[k] = 0.f;
            tile_pass<K, false>(ts, sn, xi, yi, zi, eps2, tx, ty, tz);
            tile_pass<K, true>(ts + rows - sf, sf, xi, yi, zi, eps2, tx, ty, tz);
            __syncthreads();
#pragma unroll
            for (int k = 0; k < K; ++k) {
                two_sum_fold(hx[k], lx[k], tx[k]);
                two_sum_fold(hy[k], ly[k], ty[k]);
                two_sum_fold(hz[k], lz[k], tz[k]);
            }
        }
#pragma unroll
        for (int k = 0; k < K; ++k) {
            double vx = (double)hx[k] + (double)lx[k];
            double vy = (double)hy[k] + (double)ly[k];
            double vz = (double)hz[k] + (double)lz[k];
            if (J > 1) {
                // streams 1..J-1 hand their sums to stream 0 through LDS
                if (stream > 0) {
                    red[3 * lane + 0] = vx;
                    red[3 * lane + 1] = vy;
                    red[3 * lane + 2] = vz;
                }
                __syncthreads();
                if (stream == 0) {
                    for (int q = 1; q < J; ++q) {
                        const int src = q * S + slot;
                        vx += red[3 * src + 0];
                        vy += red[3 * src + 1];
                        vz += red[3 * src + 2];
                    }
                }
                __syncthreads();
            }
            const uint32_t i = ib + slot + S * k;
            if (stream == 0 && i < n_g)
                store3<OUT64>(ax, ay, az, pidx[f + i], vx * scale, vy * scale, vz * scale);
        }
    }
    if (lane == 0) *kept_out = kept_total;
}

// One launch per blocking factor K (see k_classify), so each gets its own register budget.
// Up to K = 4 the kernel fits 128 VGPRs without spilling (4 waves per SIMD); K = 5 runs at
// 3 waves and larger K at 2.
constexpr int force_waves_per_simd(int K) { return K <= 5 ? 4 : K <= 7 ? 3 : 2; }

template <int K, int OUT64>
__global__ __launch_bounds__(64, force_waves_per_simd(K)) void k_force_f32(
    NodeArrays nd, GroupArrays gr, const uint32_t *__restrict__ ids, uint32_t n_ids,
    const uint64_t *__restrict__ off, const uint32_t *__restrict__ len, const uint32_t *__restrict__ entries,
    const double4 *__restrict__ ps, const uint32_t *__restrict__ pidx, ForceParams fp, void *ax,
    void *ay, void *az)
{
    __shared__ float4 tile[kTileF32 + 8];
    __shared__ double red[64 * 3];
    const uint32_t slot = xcd_block(blockIdx.x, gridDim.x);
    if (slot >= n_ids) return;
    const uint32_t g = ids[slot];
    const uint32_t n_g = gr.count[g], f = gr.first[g];
    const uint64_t b = off[g];
    const uint64_t Lg = len[g];
    GroupFrame F;
    F.xg0 = gr.xgx[g]; F.xg1 = gr.xgy[g]; F.xg2 = gr.xgz[g];
    F.cg0 = gr.cgx[g]; F.cg1 = gr.cgy[g]; F.cg2 = gr.cgz[g];
    F.hg0 = gr.hgx[g]; F.hg1 = gr.hgy[g]; F.hg2 = gr.hgz[g];
    F.L = fp.L;
    F.rc2 = fp.rc2;
    F.eta2 = fp.eta * fp.eta;
    F.inv_eta = fp.inv_eta;
    const float eps2 = (float)(fp.eps2 * fp.inv_eta * fp.inv_eta);
    const double scale = fp.inv_eta * fp.inv_eta;
    force_group_f32<K, OUT64>(tile, red, nd, n_g, f, entries + b, Lg, ps, pidx, F,
                              eps2, scale, ax, ay, az, fp.kept + g);
}

__global__ __launch_bounds__(256) void k_kept_stats(GroupArrays gr, uint32_t n_groups,
                                                    const uint32_t *__restrict__ kept,
                                                    unsigned long long *out)
{
    unsigned long long v = 0;
    for (uint32_t g = blockIdx.x * blockDim.x + threadIdx.x; g < n_groups;
         g += gridDim.x * blockDim.x)
        v += (unsigned long long)kept[g] * gr.count[g];
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) v += __shfl_xor(v, d, 64);
    __shared__ unsigned long long sm[4];
    if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) atomicAdd(out, sm[0] + sm[1] + sm[2] + sm[3]);
}

// Pair by pair: out[(i * n_j + j) * 3 + a] = acceleration at x_i from (x_j, m_j) with the
// FP32 pair routine of the force kernel (same relative coordinates, units and rounding),
// without the cull and without periodic images.
__global__ __launch_bounds__(256) void k_pairwise_f32(int64_t n_i, const double *__restrict__ xi,
                                                      int64_t n_j, const double *__restrict__ xj,
                                                      const double *__restrict__ mj, double xg0,
                                                      double xg1, double xg2, double inv_eta,
                                                      float eps2, double scale,
                                                      double *__restrict__ out)
{
    const int64_t total = n_i * n_j;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < total;
         q += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = q / n_j, j = q % n_j;
        const float x = (float)((xi[3 * i + 0] - xg0) * inv_eta);
        const float y = (float)((xi[3 * i + 1] - xg1) * inv_eta);
        const float z = (float)((xi[3 * i + 2] - xg2) * inv_eta);
        const float4 src = make_float4((float)((xj[3 * j + 0] - xg0) * inv_eta),
                                       (float)((xj[3 * j + 1] - xg1) * inv_eta),
                                       (float)((xj[3 * j + 2] - xg2) * inv_eta), (float)mj[j]);
        float tx = 0.f, ty = 0.f, tz = 0.f;
        pair_f32<false>(src, x, y, z, eps2, tx, ty, tz);
        out[3 * q + 0] = (double)tx * scale;
        out[3 * q + 1] = (double)ty * scale;
        out[3 * q + 2] = (double)tz * scale;
    }
}

constexpr int kClasses = 8;

// Blocking class of a group: K - 1 with K the particles per lane of force_layout.  A block
// takes kClassifyItems * 256 consecutive groups, places them with LDS atomics and reserves
// its part of each class list with one global atomic per class; the order inside a list
// does not affect results.
constexpr int kClassifyItems = 8;

__global__ __launch_bounds__(256) void k_classify(GroupArrays gr, uint32_t n_groups,
                                                  uint32_t *__restrict__ lists, uint32_t stride,
                                                  uint32_t *counts)
{
    __shared__ uint32_t s_cnt[kClasses], s_base[kClasses];
    if (threadIdx.x < kClasses) s_cnt[threadIdx.x] = 0;
    __syncthreads();
    const uint32_t base = blockIdx.x * (256u * kClassifyItems);
    int cls[kClassifyItems];
    uint32_t loc[kClassifyItems];
#pragma unroll
    for (int r = 0; r < kClassifyItems; ++r) {
        const uint32_t g = base + (uint32_t)r * 256u + threadIdx.x;
        cls[r] = -1;
        loc[r] = 0;
        if (g < n_groups) {
            int J, K;
            force_layout(gr.count[g], J, K);
            cls[r] = K - 1;
            loc[r] = atomicAdd(&s_cnt[K - 1], 1u);
        }
    }
    __syncthreads();
    if (threadIdx.x < kClasses && s_cnt[threadIdx.x])
        s_base[threadIdx.x] = atomicAdd(&counts[threadIdx.x], s_cnt[threadIdx.x]);
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kClassifyItems; ++r)
        if (cls[r] >= 0)
            lists[(uint32_t)cls[r] * stride + s_base[cls[r]] + loc[r]] =
                base + (uint32_t)r * 256u + threadIdx.x;
}

// 1/sqrt(x) in FP64 for x > 0: the hardware estimate refined by two Newton steps
// y <- y + y (1/2 - (x/2) y^2), each of which squares the relative error (to within rounding).
__device__ __forceinline__ double rsqrt_f64(double x)
{
    double y = __builtin_amdgcn_rsq(x);
    const double h = 0.5 * x;
    y = fma(y, fma(-h, y * y, 0.5), y);
    y = fma(y, fma(-h, y * y, 0.5), y);
    return y;
}

// FP64 path, one wave per group, 64 i-particles per pass.  Each tile of 64 list entries is
// culled against the group's box as in the FP32 path (a source at least r_cut from the box
// adds exactly zero) and the survivors are stored relative to x_g (nearest image, once per
// entry) in three runs: "inner" sources, whose farthest point of the box is within eta (every
// pair has R < 1: eq. (2)'s first branch only), from the front of the tile; "far" ones, at
// least eta from the box (every pair has R >= 1: the second branch only), from the back; the
// others ("near", both branches and a select) in between.  The FP64 pair evaluates both
// branches of g for a near source, so the inner run saves the second branch and the select.
// When the group's cube and cutoff fit in half the box (half side + r_cut < L/2) the
// difference of two relative positions is the nearest-image separation and the pairs need no
// wrap; otherwise the pair wraps it.  (r^2 + eps^2)^(-1/2) and r^(-1) come from
// rsqrt_f64 (r = r^2 r^(-1)); a pair at zero separation adds nothing.
constexpr int kTileF64 = 64;

enum F64Kind { kF64Near = 0, kF64Far = 1, kF64Inner = 2 };

template <int OUT64>
__global__ __launch_bounds__(64) void k_force_f64(
    NodeArrays nd, GroupArrays gr, uint32_t n_groups, const uint64_t *__restrict__ off,
    const uint32_t *__restrict__ len, const uint32_t *__restrict__ entries,
    const double4 *__restrict__ ps, const uint32_t *__restrict__ pidx, ForceParams fp, void *ax,
    void *ay, void *az)
{
    __shared__ double4 tile[kTileF64];
    const uint32_t g = xcd_block(blockIdx.x, gridDim.x);
    const int lane = threadIdx.x;
    if (g >= n_groups) return;
    const uint32_t n_g = gr.count[g], f = gr.first[g];
    const uint64_t b = off[g];
    const uint64_t Lg = len[g];
    const double L = fp.L, eps2 = fp.eps2, inv_eta = fp.inv_eta, eta2 = fp.eta * fp.eta;
    const double xg0 = gr.xgx[g], xg1 = gr.xgy[g], xg2 = gr.xgz[g];
    const double cg0 = gr.cgx[g], cg1 = gr.cgy[g], cg2 = gr.cgz[g];
    const double hg0 = gr.hgx[g], hg1 = gr.hgy[g], hg2 = gr.hgz[g];
    const double half_side = 0.5 * ldexp(L, -(int)nd.level[gr.node[g]]);
    const bool pair_wrap = !(half_side + sqrt(fp.rc2) < 0.5 * L);
    const uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;
    for (uint32_t ib = 0; ib < n_g; ib += 64) {
        const uint32_t i = ib + lane;
        const bool act = i < n_g;
        double xi = 0.0, yi = 0.0, zi = 0.0;
        if (act) {
            const double4 r = ps[f + i];
            xi = wrapd(r.x - xg0, L);
            yi = wrapd(r.y - xg1, L);
            zi = wrapd(r.z - xg2, L);
        }
        double ax_ = 0.0, ay_ = 0.0, az_ = 0.0;
        for (uint64_t jb = 0; jb < Lg; jb += kTileF64) {
            const uint64_t j = jb + lane;
            bool keep = false, far = false, inner = false;
            double4 v = make_double4(0.0, 0.0, 0.0, 0.0);
            if (j < Lg) {
                const uint32_t e = entries[b + j];
                const double4 r = (e & kCellTag) ? nd.nsrc[e & ~kCellTag] : nd.psrc[e];
                const double a0 = fabs(wrapd(r.x - cg0, L));
                const double a1 = fabs(wrapd(r.y - cg1, L));
                const double a2 = fabs(wrapd(r.z - cg2, L));
                double w0 = a0 - hg0, w1 = a1 - hg1, w2 = a2 - hg2;
                w0 = w0 > 0.0 ? w0 : 0.0;
                w1 = w1 > 0.0 ? w1 : 0.0;
                w2 = w2 > 0.0 ? w2 : 0.0;
                const double gap2 = w0 * w0 + w1 * w1 + w2 * w2;
                const double e0 = a0 + hg0, e1 = a1 + hg1, e2 = a2 + hg2;
                keep = gap2 < fp.rc2;
                far = gap2 >= eta2;
                inner = e0 * e0 + e1 * e1 + e2 * e2 < eta2;
                v = make_double4(wrapd(r.x - xg0, L), wrapd(r.y - xg1, L), wrapd(r.z - xg2, L),
                                 r.w);
            }
            const uint64_t mi = __ballot(keep && inner), mn = __ballot(keep && !far && !inner),
                           mf = __ballot(keep && far);
            const int ni = __popcll(mi), nn = __popcll(mn), nf = __popcll(mf);
            if (keep) {
                if (far)
                    tile[kTileF64 - 1 - __popcll(mf & lt)] = v;
                else if (inner)
                    tile[__popcll(mi & lt)] = v;
                else
                    tile[ni + __popcll(mn & lt)] = v;
            }
            __syncthreads();
#define TPM_F64_PAIRS(KIND, WRAP, T0, T1)                                                       \
    for (int t = (T0); t < (T1); ++t) {                                                        \
        const double4 s = tile[t];                                                             \
        double dx = s.x - xi, dy = s.y - yi, dz = s.z - zi;                                    \
        if (WRAP) {                                                                            \
            dx = wrapd(dx, L);                                                                 \
            dy = wrapd(dy, L);                                                                 \
            dz = wrapd(dz, L);                                                                 \
        }                                                                                      \
        const double r2 = dx * dx + dy * dy + dz * dz;                                         \
        const double is = rsqrt_f64(r2 + eps2);                                                \
        const double R = r2 * rsqrt_f64(r2) * inv_eta;                                         \
        const double g = KIND == kF64Far     ? g_far_f64(R)                                   \
                         : KIND == kF64Inner ? g_in_f64(R)                                    \
                                             : g_p3m_f64(R);                                  \
        double fm = s.w * g * (is * is * is);                                                  \
        fm = r2 > 0.0 ? fm : 0.0;                                                              \
        ax_ += fm * dx;                                                                        \
        ay_ += fm * dy;                                                                        \
        az_ += fm * dz;                                                                        \
    }
            if (pair_wrap) {
                TPM_F64_PAIRS(kF64Inner, true, 0, ni)
                TPM_F64_PAIRS(kF64Near, true, ni, ni + nn)
                TPM_F64_PAIRS(kF64Far, true, kTileF64 - nf, kTileF64)
            } else {
                TPM_F64_PAIRS(kF64Inner, false, 0, ni)
                TPM_F64_PAIRS(kF64Near, false, ni, ni + nn)
                TPM_F64_PAIRS(kF64Far, false, kTileF64 - nf, kTileF64)
            }
#undef TPM_F64_PAIRS
            __syncthreads();
        }
        if (act) store3<OUT64>(ax, ay, az, pidx[f + i], ax_, ay_, az_);
    }
}

} // namespace

void launch_classify(GroupArrays gr, uint32_t n_groups, uint32_t *lists, uint32_t stride,
                     uint32_t *counts, hipStream_t s)
{
    fill_u32(counts, kClasses, 0u, s);
    if (!n_groups) return;
    const unsigned b = (n_groups + 256u * kClassifyItems - 1) / (256u * kClassifyItems);
    k_classify<<<b, 256, 0, s>>>(gr, n_groups, lists, stride, counts);
}

void launch_force_f32(NodeArrays nd, GroupArrays gr, const uint32_t *lists, uint32_t stride,
                      const uint32_t *class_counts, const uint64_t *off, const uint32_t *len,
                      const uint32_t *entries, const double4 *ps, const uint32_t *pidx,
                      ForceParams fp, void *ax, void *ay, void *az, int out_prec,
                      const hipStream_t *streams, int n_streams)
{
    int next = 0;
#define TPM_LAUNCH(KK)                                                                         \
    if (class_counts[KK - 1]) {                                                                \
        const uint32_t *ids = lists + (size_t)(KK - 1) * stride;                               \
        hipStream_t s = streams[next++ % n_streams];                                           \
        if (out_prec)                                                                          \
            k_force_f32<KK, 1><<<class_counts[KK - 1], 64, 0, s>>>(                            \
                nd, gr, ids, class_counts[KK - 1], off, len, entries, ps, pidx, fp, ax, \
                ay, az);                                                                       \
        else                                                                                   \
            k_force_f32<KK, 0><<<class_counts[KK - 1], 64, 0, s>>>(                            \
                nd, gr, ids, class_counts[KK - 1], off, len, entries, ps, pidx, fp, ax, \
                ay, az);                                                                       \
    }
    TPM_LAUNCH(8)
    TPM_LAUNCH(7)
    TPM_LAUNCH(6)
    TPM_LAUNCH(5)
    TPM_LAUNCH(4)
    TPM_LAUNCH(3)
    TPM_LAUNCH(2)
    TPM_LAUNCH(1)
#undef TPM_LAUNCH
}

void launch_pairwise_f32(int64_t n_i, const double *xi, int64_t n_j, const double *xj,
                         const double *mj, const double *xg, double eta, double eps,
                         double *out, hipStream_t s)
{
    const double inv_eta = 1.0 / eta;
    const int64_t total = n_i * n_j;
    int64_t b = (total + 255) / 256;
    k_pairwise_f32<<<(unsigned)(b < 65536 ? (b > 0 ? b : 1) : 65536), 256, 0, s>>>(
        n_i, xi, n_j, xj, mj, xg[0], xg[1], xg[2], inv_eta, (float)(eps * eps * inv_eta * inv_eta),
        inv_eta * inv_eta, out);
}

void launch_kept_stats(GroupArrays gr, uint32_t n_groups, const uint32_t *kept,
                       unsigned long long *out, hipStream_t s)
{
    fill_u64((uint64_t *)out, 1, 0ull, s);
    if (!n_groups) return;
    unsigned b = (n_groups + 255) / 256;
    k_kept_stats<<<b < 256 ? b : 256, 256, 0, s>>>(gr, n_groups, kept, out);
}

void launch_force_f64(NodeArrays nd, GroupArrays gr, uint32_t n_groups, const uint64_t *off,
                      const uint32_t *len, const uint32_t *entries, const double4 *ps, const uint32_t *pidx,
                      ForceParams fp, void *ax, void *ay, void *az, int out_prec,
                      hipStream_t s)
{
    if (!n_groups) return;
    if (out_prec)
        k_force_f64<1><<<n_groups, 64, 0, s>>>(nd, gr, n_groups, off, len, entries, ps, pidx, fp,
                                              ax, ay, az);
    else
        k_force_f64<0><<<n_groups, 64, 0, s>>>(nd, gr, n_groups, off, len, entries, ps, pidx, fp,
                                              ax, ay, az);
}

} // namespace tpm
