// Short-range pair force over the interaction lists (Section 2.1 eq. 1 with the cutoff
// g_P3M of eq. 2 and Plummer softening of Section 2.4):
//
//   a_i += m_j d g(|d| / eta) / (|d|^2 + eps^2)^(3/2),   d = x_j - x_i.
//
// One 64-lane wavefront per group: the group's i-particles sit in registers and its list is
// streamed through LDS in tiles; lanes of one stream read the same tile entry (an LDS
// broadcast) and accumulate in registers.  List entries whose source lies at least r_cut from
// the group's bounding box are dropped while a tile is loaded (every pair they form adds
// exactly zero).
//
// FP32 path (Section 3.1.1): positions are passed relative to the group's cube centre x_g,
// x_i - x_g and wrap(x_j - x_g), each difference taken in FP64 and then rounded to FP32, so
// the rounding error of the subtraction scales with the group size, not the box.  The pair
// law is read from a per-box table of cubic pieces (see the FP32 section).  The per-tile FP32
// partial sums are folded into an FP32 (hi, lo) pair with TwoSum.  Persistent workgroups
// take the groups from per-XCD queues, the heaviest groups first.  Each particle's result
// leaves the kernels as one record in the caller's order, which a last pass splits into the
// output arrays or applies as a kick.
//
// FP64 path: the same relative coordinates in FP64 (nearest image once per entry, or per pair
// when the group's cube plus r_cut reaches half the box), (r^2 + eps^2)^(-1/2) and r^(-1)
// from the hardware estimate refined by two Newton steps, and eq. (2) evaluated directly in a
// form with no cancellation: for R < 1,
//   g = 1 + R^3 (-8/5 + R^2 (8/5 + R (-1/2 + R (-12/35 + 3R/20)))),
// and for R >= 1, g = max(2 - R, 0)^5 (7R^3 + 22R^2 + 10R + 4) / 140 (zero from R = 2 on).
// Both are eq. (2) rearranged.
#include "common.hpp"

#include <cmath>
#include <utility>
#include <vector>

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

// The force kernels leave one record per particle, in the caller's order: float4 (ax, ay, az,
// 0) for float results, double4 for double results and for the kick.  The caller's order is
// arbitrary, so each store lands in its own 32-byte HBM sector: one 16- or 32-byte record costs
// one sector where three 4- or 8-byte component stores cost three.  k_force_out then walks the
// records in order and splits them into the caller's three arrays (kOutF32, kOutF64) or adds dt
// times them to double velocities (kOutKick: the kick of Section 2.2 step 5 taken with the
// short-range force as soon as it is known), each product and sum rounded on its own.
enum { kOutF32 = 0, kOutF64 = 1, kOutKick = 2 };

template <int REC64>
__device__ __forceinline__ void store_rec(void *rec, uint32_t i, double vx, double vy, double vz)
{
    if (REC64)
        ((double4 *)rec)[i] = make_double4(vx, vy, vz, 0.0);
    else
        ((float4 *)rec)[i] = make_float4((float)vx, (float)vy, (float)vz, 0.0f);
}

// FP32 path.  Lengths are in units of r_cut = 2 eta, and the pair law is
//   a_i = (1/r_cut^2) sum_j m_j d'_ij G(|d'_ij|^2),   G(s) = g(2 sqrt(s)) / (s + (eps/r_cut)^2)^(3/2),
// so the 1/r_cut^2 is applied once per particle and the cutoff is at s = 1.  G is read from a
// table of cubic pieces built on the host for the box's eps/r_cut (build_force_table): the
// variable u = s + c (c a power of two far below (eps/r_cut)^2, added inside the fused sum
// of squares, whose result is clamped to 1) is cut into 32 pieces per octave by its own bit
// pattern, so the piece index is the exponent and top five mantissa bits of u and the
// position inside the piece is the remaining 18 mantissa bits, both exact.  The table holds
// H = G / (1 - s)^4 (the power of 1 - s takes most of eq. 2's fifth-order zero at the
// cutoff, so the cubics keep G's relative accuracy there); u = 1 (every R >= 2, by the clamp)
// falls on a zero piece.  A pair costs 21 vector instructions and one LDS read and needs no
// square root, reciprocal square root or branch.
//
// One tile takes up to kTileF32 list entries.  Each lane examines kTileF32 / 64 of them and
// drops those whose source is at least r_cut from the group's bounding box: every pair they
// would form is at least r_cut apart and adds exactly zero (g = 0 for R >= 2).  Survivors are
// compacted in list order and dealt to the J streams: survivor e goes to stream e % J, row
// e / J.  Rows past the last survivor of a stream are zero-mass padding (they add exactly 0).
constexpr int kTileF32 = 256;
constexpr int kTileRounds = kTileF32 / 64;
constexpr int kForceWaves = 4; // waves per workgroup; each runs its own groups, sharing the table

struct GroupFrame {
    double xg0, xg1, xg2;   // x_g, origin of the relative coordinates
    double cg0, cg1, cg2;   // bbox centre
    double hg0, hg1, hg2;   // bbox half size
    double L, rc2, inv_len; // inv_len = 1 / r_cut, the FP32 path's length unit
};

// The LDS writes of this wave are complete before any of its lanes reads LDS again (the
// waves of a workgroup work on different groups, so a workgroup barrier is not wanted).
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_s_waitcnt(0xc07f); // lgkmcnt(0); vector memory counters untouched
    __builtin_amdgcn_wave_barrier();
}

// The list entries of the tile starting at jb (jb < Lg), one per lane and round.  Slots past
// the list's end read its last entry and are dropped by load_tile_f32.  The caller issues
// these reads one tile ahead, so they are in flight while the previous tile is evaluated.
__device__ __forceinline__ void fetch_entries(const uint32_t *__restrict__ list, uint64_t jb,
                                              uint64_t Lg, uint32_t *ent)
{
    const int lane = __lane_id();
#pragma unroll
    for (int r = 0; r < kTileRounds; ++r) {
        const uint64_t j = jb + (uint64_t)(r * 64 + lane);
        ent[r] = list[j < Lg ? j : Lg - 1];
    }
}

// Culls and packs one tile; returns the number of survivors (the same on every lane).  WRAP
// = false for a group whose bounding box, grown by r_cut, lies inside [0, L) on every axis:
// then a source within r_cut of the box is its own nearest image, and a source whose nearest
// image lies across the boundary is at least r_cut from the box without the wrap as with it,
// so no coordinate needs wrapping.
template <bool WRAP>
__device__ __forceinline__ double wrapc(double v, double L)
{
    return WRAP ? wrapd(v, L) : v;
}

template <bool WRAP>
__device__ __forceinline__ int load_tile_f32(float4 *tile, const uint32_t *ent, uint64_t jb,
                                             uint64_t Lg, int J, int lgJ, NodeArrays nd,
                                             const GroupFrame &F)
{
    constexpr int kR = kTileRounds;
    const int lane = __lane_id();
    const int rows = kTileF32 >> lgJ;
    const uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;
    int n = 0;
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
        bool keep = false;
        float4 v;
        if (j < Lg) {
            const double4 src = srcs[r];
            const double sx = src.x, sy = src.y, sz = src.z, sm = src.w;
            double w0 = fabs(wrapc<WRAP>(sx - F.cg0, F.L)) - F.hg0;
            double w1 = fabs(wrapc<WRAP>(sy - F.cg1, F.L)) - F.hg1;
            double w2 = fabs(wrapc<WRAP>(sz - F.cg2, F.L)) - F.hg2;
            w0 = w0 > 0.0 ? w0 : 0.0;
            w1 = w1 > 0.0 ? w1 : 0.0;
            w2 = w2 > 0.0 ? w2 : 0.0;
            keep = w0 * w0 + w1 * w1 + w2 * w2 < F.rc2;
            v = make_float4((float)(wrapc<WRAP>(sx - F.xg0, F.L) * F.inv_len),
                            (float)(wrapc<WRAP>(sy - F.xg1, F.L) * F.inv_len),
                            (float)(wrapc<WRAP>(sz - F.xg2, F.L) * F.inv_len), (float)sm);
        }
        const uint64_t mk = __ballot(keep);
        if (keep) {
            const int e = n + (int)__popcll(mk & lt);
            tile[(e & (J - 1)) * rows + (e >> lgJ)] = v;
        }
        n += (int)__popcll(mk);
    }
    // zero the padding slots of the last row
    const int e = n + lane;
    if (lane < J && e < ((n + J - 1) >> lgJ) << lgJ)
        tile[(e & (J - 1)) * rows + (e >> lgJ)] = make_float4(0.f, 0.f, 0.f, 0.f);
    return __builtin_amdgcn_readfirstlane(n);
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

struct TabView {
    const float4 *tb; // the table in LDS, offset so that tb[bits(u) >> kTabShift] is u's piece
    float c;
    float c1;         // 1 + c
};

// One pair from the table: s = (x_j', m_j), lane particle (xi, yi, zi), all in units of
// r_cut.  21 vector instructions.
__device__ __forceinline__ void pair_f32(const float4 s, float xi, float yi, float zi,
                                         const TabView &T, float &tx, float &ty, float &tz)
{
    const float dx = s.x - xi, dy = s.y - yi, dz = s.z - zi;
    // u = min(s + c, 1): the clamp is an output modifier of the last fma
    const float u = __builtin_amdgcn_fmed3f(fmaf(dx, dx, fmaf(dy, dy, fmaf(dz, dz, T.c))), 0.0f,
                                            1.0f);
    const uint32_t b = __float_as_uint(u);
    // the piece index as a separate shift (an instruction the compiler does not merge with
    // the address scaling, which then folds into one shift-and-add)
    uint32_t k;
    asm("v_lshrrev_b32 %0, 18, %1" : "=v"(k) : "v"(b));
    static_assert(kTabShift == 18, "the shift above is kTabShift");
    const float4 q = T.tb[k];
    // position inside the piece: the low mantissa bits as a float x in [1, 2)
    const float x = __uint_as_float(((b << kTabSegBits) & 0x007fffffu) | 0x3f800000u);
    const float H = fmaf(fmaf(fmaf(q.w, x, q.z), x, q.y), x, q.x);
    // G = (1 - s)^4 H; 1 - s = (1 + c) - u is exact for u >= 1/2
    const float w = T.c1 - u, w2 = w * w;
    const float fm = s.w * ((w2 * w2) * H);
    tx = fmaf(fm, dx, tx);
    ty = fmaf(fm, dy, ty);
    tz = fmaf(fm, dz, tz);
}

// steps rows of a stream's tile run, starting at ts, against the lane's K i-particles.
template <int K>
__device__ __forceinline__ void tile_pass(const float4 *ts, int steps, const float *xi,
                                          const float *yi, const float *zi, const TabView &T,
                                          float *tx, float *ty, float *tz)
{
    int t = 0;
    if (K < 4) { // two rows per iteration; larger K has enough independent pairs per row
        for (; t + 2 <= steps; t += 2) {
            const float4 s0 = ts[t], s1 = ts[t + 1];
#pragma unroll
            for (int k = 0; k < K; ++k) {
                pair_f32(s0, xi[k], yi[k], zi[k], T, tx[k], ty[k], tz[k]);
                pair_f32(s1, xi[k], yi[k], zi[k], T, tx[k], ty[k], tz[k]);
            }
        }
    }
    for (; t < steps; ++t) {
        const float4 s0 = ts[t];
#pragma unroll
        for (int k = 0; k < K; ++k) pair_f32(s0, xi[k], yi[k], zi[k], T, tx[k], ty[k], tz[k]);
    }
}

// Whether the next tile's list entries are read while the current tile is evaluated: only
// where the four extra registers do not push the class past its register budget.
__host__ __device__ constexpr bool force_prefetch(int K) { return K <= 4 || K == 6 || K == 8; }

// One group on one wave in the layout of force_layout (K i-particles per lane, J streams,
// each stream taking every J-th surviving source); the J partial sums are added at the end
// in stream order.  tile: this wave's kTileF32 LDS slots (also used for that reduction).
template <int K, int REC64, bool WRAP>
__device__ __forceinline__ void force_group_f32(float4 *tile, const TabView &T, NodeArrays nd,
                                                uint32_t n_g, uint32_t f, const uint32_t *list,
                                                uint64_t Lg, const double4 *__restrict__ ps,
                                                const uint32_t *__restrict__ pidx,
                                                const GroupFrame &F, double scale, void *rec,
                                                uint32_t *kept_out)
{
    const int lane = __lane_id();
    int J, Kl;
    force_layout(n_g, J, Kl);
    (void)Kl; // equals K: the group was classified with the same layout
    const int S = 64 / J;
    const int lgJ = J == 1 ? 0 : J == 2 ? 1 : J == 4 ? 2 : 3;
    const int slot = lane % S, stream = lane / S;
    const int rows = kTileF32 >> lgJ;
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
                xi[k] = (float)((r.x - F.xg0) * F.inv_len);
                yi[k] = (float)((r.y - F.xg1) * F.inv_len);
                zi[k] = (float)((r.z - F.xg2) * F.inv_len);
            }
            hx[k] = hy[k] = hz[k] = lx[k] = ly[k] = lz[k] = 0.f;
        }
        uint32_t ent[kTileRounds];
        if (force_prefetch(K) && Lg) fetch_entries(list, 0, Lg, ent);
        for (uint64_t jb = 0; jb < Lg; jb += kTileF32) {
            if (!force_prefetch(K)) fetch_entries(list, jb, Lg, ent);
            const int nt = load_tile_f32<WRAP>(tile, ent, jb, Lg, J, lgJ, nd, F);
            kept_total += (uint32_t)nt;
            wave_lds_sync();
            if (force_prefetch(K) && jb + kTileF32 < Lg)
                fetch_entries(list, jb + kTileF32, Lg, ent);
            const int steps = (nt + J - 1) >> lgJ; // the same on every lane
            float tx[K], ty[K], tz[K];
#pragma unroll
            for (int k = 0; k < K; ++k) tx[k] = ty[k] = tz[k] = 0.f;
            tile_pass<K>(tile + stream * rows, steps, xi, yi, zi, T, tx, ty, tz);
            wave_lds_sync();
#pragma unroll
            for (int k = 0; k < K; ++k) {
                two_sum_fold(hx[k], lx[k], tx[k]);
                two_sum_fold(hy[k], ly[k], ty[k]);
                two_sum_fold(hz[k], lz[k], tz[k]);
            }
        }
        double *red = reinterpret_cast<double *>(tile); // 64 x 3 doubles fit the tile
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
                wave_lds_sync();
                if (stream == 0) {
                    for (int q = 1; q < J; ++q) {
                        const int src = q * S + slot;
                        vx += red[3 * src + 0];
                        vy += red[3 * src + 1];
                        vz += red[3 * src + 2];
                    }
                }
                wave_lds_sync();
            }
            const uint32_t i = ib + slot + S * k;
            if (stream == 0 && i < n_g)
                store_rec<REC64>(rec, pidx[f + i], vx * scale, vy * scale, vz * scale);
        }
    }
    *kept_out = kept_total; // the same value on every lane
}

// One kernel per blocking factor K, so each gets its own register budget.  Up to K = 4 the
// kernel fits 128 VGPRs without spilling (4 waves per SIMD); K = 5 runs at 4, 6-7 at 3 and 8
// at 2.
constexpr int force_waves_per_simd(int K) { return K <= 5 ? 4 : K <= 7 ? 3 : 2; }

// Persistent: each workgroup copies the table into LDS once and its waves then take groups
// from the class's queues until all are empty.  The class's groups are split into kXcds
// parts, each a contiguous range of groups in key order (neighbouring groups share sources),
// sorted by decreasing cost n_g L_g (the longest lists first, so the last groups to finish
// are short).  A workgroup starts on the part of its own XCD (workgroups are dealt to the
// XCDs round-robin by block index) and then takes from the others'.
template <int K, int REC64>
__global__ __launch_bounds__(64 * kForceWaves, force_waves_per_simd(K)) void k_force_f32(
    NodeArrays nd, GroupArrays gr, const uint32_t *__restrict__ ids,
    const uint32_t *__restrict__ part_start, uint32_t *queue, const uint64_t *__restrict__ off,
    const uint32_t *__restrict__ len, const uint32_t *__restrict__ entries,
    const double4 *__restrict__ ps, const uint32_t *__restrict__ pidx, ForceParams fp,
    ForceTable ft, void *rec)
{
    extern __shared__ float4 smem[];
    for (uint32_t i = threadIdx.x; i < ft.entries; i += blockDim.x) smem[i] = ft.coef[i];
    __syncthreads();
    const TabView T{smem - ft.base, ft.c, 1.0f + ft.c};
    float4 *tile = smem + ft.entries + (threadIdx.x >> 6) * kTileF32;
    const uint32_t lane = __lane_id();
    GroupFrame F;
    F.L = fp.L;
    F.rc2 = fp.rc2;
    F.inv_len = 0.5 * fp.inv_eta; // 1 / r_cut
    const double scale = F.inv_len * F.inv_len;
    const uint32_t xcd = blockIdx.x % kXcds;
    for (uint32_t p = 0; p < kXcds; ++p) {
        const uint32_t part = (xcd + p) % kXcds;
        const uint32_t lo = part_start[part], size = part_start[part + 1] - lo;
        for (;;) {
            // One slot per wave: every lane takes part in the atomic (lane 0 adds 1, the others
            // 0) and the wave reads lane 0's result, so no branch depends on the lane here.
            const uint32_t q =
                __builtin_amdgcn_readfirstlane(atomicAdd(&queue[part], lane == 0 ? 1u : 0u));
            if (q >= size) break;
            const uint32_t g = ids[lo + q];
            F.xg0 = gr.xgx[g]; F.xg1 = gr.xgy[g]; F.xg2 = gr.xgz[g];
            F.cg0 = gr.cgx[g]; F.cg1 = gr.cgy[g]; F.cg2 = gr.cgz[g];
            F.hg0 = gr.hgx[g]; F.hg1 = gr.hgy[g]; F.hg2 = gr.hgz[g];
            const double rc = fp.rc * (1.0 + 0x1p-10); // clear of rounding at the boundary
            const bool interior = gr.lox[g] - rc >= 0.0 && gr.hix[g] + rc < fp.L &&
                                  gr.loy[g] - rc >= 0.0 && gr.hiy[g] + rc < fp.L &&
                                  gr.loz[g] - rc >= 0.0 && gr.hiz[g] + rc < fp.L;
            if (interior)
                force_group_f32<K, REC64, false>(tile, T, nd, gr.count[g], gr.first[g],
                                                 entries + off[g], len[g], ps, pidx, F, scale,
                                                 rec, fp.kept + g);
            else
                force_group_f32<K, REC64, true>(tile, T, nd, gr.count[g], gr.first[g],
                                                entries + off[g], len[g], ps, pidx, F, scale,
                                                rec, fp.kept + g);
        }
    }
}

// k_force_f32 over several boxes (float4 records): the workgroup takes the boxes in order
// and, within each, the class's queues as above.  The tiles sit at the front of LDS and the
// table after them; at a box whose table differs from the one loaded, the workgroup waits
// for its waves to finish the previous box and copies the new table.  Every wave sees the
// same boxes, class sizes and table ids, so all reach the same barriers.
template <int K>
__global__ __launch_bounds__(64 * kForceWaves, force_waves_per_simd(K)) void k_force_f32_multi(
    const ForceBox *__restrict__ bx, int nb)
{
    extern __shared__ float4 smem[];
    float4 *tile = smem + (threadIdx.x >> 6) * kTileF32;
    float4 *tab = smem + kForceWaves * kTileF32;
    const uint32_t lane = __lane_id();
    const uint32_t xcd = blockIdx.x % kXcds;
    uint64_t loaded = 0;
    bool have = false;
    for (int b = 0; b < nb; ++b) {
        const ForceBox &B = bx[b];
        uint32_t *cls = B.cls;
        if (cls[kClsCounts + K - 1] == 0) continue;
        if (!have || B.tab_id != loaded) {
            __syncthreads(); // the previous table is no longer read
            for (uint32_t i = threadIdx.x; i < B.ft.entries; i += blockDim.x) tab[i] = B.ft.coef[i];
            __syncthreads();
            loaded = B.tab_id;
            have = true;
        }
        const TabView T{tab - B.ft.base, B.ft.c, 1.0f + B.ft.c};
        GroupFrame F;
        F.L = B.fp.L;
        F.rc2 = B.fp.rc2;
        F.inv_len = 0.5 * B.fp.inv_eta; // 1 / r_cut
        const double scale = F.inv_len * F.inv_len;
        const double rc = B.fp.rc * (1.0 + 0x1p-10);
        const uint32_t *part_start = cls + kClsStarts + (K - 1) * (kXcds + 1);
        uint32_t *queue = cls + kClsQueue + (K - 1) * kXcds;
        const GroupArrays &gr = B.gr;
        for (uint32_t p = 0; p < kXcds; ++p) {
            const uint32_t part = (xcd + p) % kXcds;
            const uint32_t lo = part_start[part], size = part_start[part + 1] - lo;
            for (;;) {
                const uint32_t q =
                    __builtin_amdgcn_readfirstlane(atomicAdd(&queue[part], lane == 0 ? 1u : 0u));
                if (q >= size) break;
                const uint32_t g = cls[lo + q];
                F.xg0 = gr.xgx[g]; F.xg1 = gr.xgy[g]; F.xg2 = gr.xgz[g];
                F.cg0 = gr.cgx[g]; F.cg1 = gr.cgy[g]; F.cg2 = gr.cgz[g];
                F.hg0 = gr.hgx[g]; F.hg1 = gr.hgy[g]; F.hg2 = gr.hgz[g];
                const bool interior = gr.lox[g] - rc >= 0.0 && gr.hix[g] + rc < F.L &&
                                      gr.loy[g] - rc >= 0.0 && gr.hiy[g] + rc < F.L &&
                                      gr.loz[g] - rc >= 0.0 && gr.hiz[g] + rc < F.L;
                if (interior)
                    force_group_f32<K, 0, false>(tile, T, B.nd, gr.count[g], gr.first[g],
                                                 B.entries + B.off[g], B.len[g], B.ps, B.pidx,
                                                 F, scale, B.rec, B.fp.kept + g);
                else
                    force_group_f32<K, 0, true>(tile, T, B.nd, gr.count[g], gr.first[g],
                                                B.entries + B.off[g], B.len[g], B.ps, B.pidx,
                                                F, scale, B.rec, B.fp.kept + g);
            }
        }
    }
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
// FP32 pair routine of the force kernel (same relative coordinates, units, table and
// rounding), without the cull and without periodic images.
__global__ __launch_bounds__(256) void k_pairwise_f32(int64_t n_i, const double *__restrict__ xi,
                                                      int64_t n_j, const double *__restrict__ xj,
                                                      const double *__restrict__ mj, double xg0,
                                                      double xg1, double xg2, double inv_len,
                                                      ForceTable ft, double scale,
                                                      double *__restrict__ out)
{
    const TabView T{ft.coef - ft.base, ft.c, 1.0f + ft.c};
    const int64_t total = n_i * n_j;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < total;
         q += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = q / n_j, j = q % n_j;
        const float x = (float)((xi[3 * i + 0] - xg0) * inv_len);
        const float y = (float)((xi[3 * i + 1] - xg1) * inv_len);
        const float z = (float)((xi[3 * i + 2] - xg2) * inv_len);
        const float4 src = make_float4((float)((xj[3 * j + 0] - xg0) * inv_len),
                                       (float)((xj[3 * j + 1] - xg1) * inv_len),
                                       (float)((xj[3 * j + 2] - xg2) * inv_len), (float)mj[j]);
        float tx = 0.f, ty = 0.f, tz = 0.f;
        pair_f32(src, x, y, z, T, tx, ty, tz);
        out[3 * q + 0] = (double)tx * scale;
        out[3 * q + 1] = (double)ty * scale;
        out[3 * q + 2] = (double)tz * scale;
    }
}

// Classes and queues of the FP32 force.  Group g belongs to class q = K - 1 (K of its lane
// layout), to XCD part p = floor(8 g / G) (contiguous key ranges) and to a cost bucket: the
// octave of n_g L_g for heavy groups (at least 2^kHeavyCost pairs, which take a wave a
// large part of a millisecond), one bucket for all others.  The bins (q, p, bucket) are laid
// out with the costliest bucket first, so each part of each class lists its heavy groups
// longest first and then the rest in about key order (consecutive groups share sources
// through the XCD's L2).  Three passes: count the bins, scan them into cursors and part
// starts, scatter.  Blocks take kClassifyItems * 256 consecutive groups and aggregate their
// bins in LDS first.
constexpr int kClassifyItems = 8;
constexpr int kCostBuckets = 64;
constexpr uint32_t kHeavyCost = 17;
constexpr int kBins = kForceClasses * kXcds * kCostBuckets;

__device__ __forceinline__ uint32_t cost_bin(uint32_t g, uint32_t n_groups, uint32_t n_g,
                                             uint32_t L_g)
{
    int J, K;
    force_layout(n_g, J, K);
    const uint32_t part = (uint32_t)(((uint64_t)g * kXcds) / n_groups);
    const uint64_t cost = (uint64_t)n_g * L_g;
    uint32_t b = 0;
    if (cost >= (1ull << kHeavyCost)) {
        const uint32_t lg = 63u - (uint32_t)__clzll((long long)cost);
        b = lg - kHeavyCost + 1;
        b = b < kCostBuckets ? b : kCostBuckets - 1;
    }
    return ((uint32_t)(K - 1) * kXcds + part) * kCostBuckets + (kCostBuckets - 1 - b);
}

__global__ __launch_bounds__(256) void k_class_count(GroupArrays gr, uint32_t n_groups,
                                                     const uint32_t *__restrict__ len,
                                                     uint32_t *hist)
{
    __shared__ uint32_t s_cnt[kBins];
    for (int i = threadIdx.x; i < kBins; i += 256) s_cnt[i] = 0;
    __syncthreads();
    const uint32_t base = blockIdx.x * (256u * kClassifyItems);
#pragma unroll
    for (int r = 0; r < kClassifyItems; ++r) {
        const uint32_t g = base + (uint32_t)r * 256u + threadIdx.x;
        if (g < n_groups) atomicAdd(&s_cnt[cost_bin(g, n_groups, gr.count[g], len[g])], 1u);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kBins; i += 256)
        if (s_cnt[i]) atomicAdd(&hist[i], s_cnt[i]);
}

// One thread per class: bins to cursors (in place), part starts and the class size.
__global__ void k_class_scan(uint32_t *cls, uint32_t stride)
{
    const uint32_t q = threadIdx.x;
    if (q >= kForceClasses) return;
    uint32_t *hist = cls + kClsBins + q * kXcds * kCostBuckets;
    uint32_t *start = cls + kClsStarts + q * (kXcds + 1);
    const uint32_t origin = kClsLists + q * stride;
    uint32_t pos = origin;
    for (int p = 0; p < kXcds; ++p) {
        start[p] = pos;
        for (int b = 0; b < kCostBuckets; ++b) {
            const uint32_t c = hist[p * kCostBuckets + b];
            hist[p * kCostBuckets + b] = pos;
            pos += c;
        }
    }
    start[kXcds] = pos;
    cls[kClsCounts + q] = pos - origin;
}

__global__ __launch_bounds__(256) void k_class_scatter(GroupArrays gr, uint32_t n_groups,
                                                       const uint32_t *__restrict__ len,
                                                       uint32_t *cls)
{
    __shared__ uint32_t s_cnt[kBins];
    for (int i = threadIdx.x; i < kBins; i += 256) s_cnt[i] = 0;
    __syncthreads();
    const uint32_t base = blockIdx.x * (256u * kClassifyItems);
    uint32_t bin[kClassifyItems], loc[kClassifyItems];
#pragma unroll
    for (int r = 0; r < kClassifyItems; ++r) {
        const uint32_t g = base + (uint32_t)r * 256u + threadIdx.x;
        bin[r] = ~0u;
        if (g < n_groups) {
            bin[r] = cost_bin(g, n_groups, gr.count[g], len[g]);
            loc[r] = atomicAdd(&s_cnt[bin[r]], 1u);
        }
    }
    __syncthreads();
    // this block's run of each bin
    for (int i = threadIdx.x; i < kBins; i += 256)
        if (s_cnt[i]) s_cnt[i] = atomicAdd(&cls[kClsBins + i], s_cnt[i]);
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kClassifyItems; ++r)
        if (bin[r] != ~0u) cls[s_cnt[bin[r]] + loc[r]] = base + (uint32_t)r * 256u + threadIdx.x;
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

template <int REC64>
__global__ __launch_bounds__(64) void k_force_f64(
    NodeArrays nd, GroupArrays gr, uint32_t n_groups, const uint64_t *__restrict__ off,
    const uint32_t *__restrict__ len, const uint32_t *__restrict__ entries,
    const double4 *__restrict__ ps, const uint32_t *__restrict__ pidx, ForceParams fp,
    void *rec)
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
    uint32_t kept_total = 0;
    for (uint32_t ib = 0; ib < n_g; ib += 64) {
        const uint32_t i = ib + lane;
        const bool act = i < n_g;
        kept_total = 0;
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
            kept_total += (uint32_t)(ni + nn + nf);
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
        if (act) store_rec<REC64>(rec, pidx[f + i], ax_, ay_, az_);
    }
    if (lane == 0) fp.kept[g] = kept_total;
}

// The records in the caller's order, split into three arrays or applied as a kick (modes as
// for store_rec; records are float4 for kOutF32, double4 otherwise).
template <int MODE>
__global__ __launch_bounds__(256) void k_force_out(const void *__restrict__ rec, int64_t n,
                                                   void *ax, void *ay, void *az, double dt)
{
    // the kick's product and sum are rounded separately: no fused multiply-add here (the
    // rest of this file contracts)
#pragma clang fp contract(off)
    for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < n;
         j += (int64_t)gridDim.x * 256) {
        if (MODE == kOutF32) {
            const float4 r = ((const float4 *)rec)[j];
            ((float *)ax)[j] = r.x;
            ((float *)ay)[j] = r.y;
            ((float *)az)[j] = r.z;
        } else {
            const double4 r = ((const double4 *)rec)[j];
            if (MODE == kOutF64) {
                ((double *)ax)[j] = r.x;
                ((double *)ay)[j] = r.y;
                ((double *)az)[j] = r.z;
            } else {
                double *const vx = (double *)ax, *const vy = (double *)ay, *const vz = (double *)az;
                vx[j] = vx[j] + dt * r.x;
                vy[j] = vy[j] + dt * r.y;
                vz[j] = vz[j] + dt * r.z;
            }
        }
    }
}

} // namespace

void launch_classify(GroupArrays gr, uint32_t n_groups, const uint32_t *len, uint32_t *cls,
                     uint32_t stride, hipStream_t s)
{
    fill_u32(cls, kClsLists, 0u, s);
    if (!n_groups) return;
    const unsigned b = (n_groups + 256u * kClassifyItems - 1) / (256u * kClassifyItems);
    k_class_count<<<b, 256, 0, s>>>(gr, n_groups, len, cls + kClsBins);
    k_class_scan<<<1, 64, 0, s>>>(cls, stride);
    k_class_scatter<<<b, 256, 0, s>>>(gr, n_groups, len, cls);
}

void launch_force_f32(NodeArrays nd, GroupArrays gr, uint32_t *cls, const uint32_t *class_counts,
                      const uint64_t *off, const uint32_t *len, const uint32_t *entries,
                      const double4 *ps, const uint32_t *pidx, ForceParams fp, ForceTable ft,
                      void *rec, int rec64, int n_cu, const hipStream_t *streams,
                      int n_streams)
{
    const size_t lds = ((size_t)ft.entries + (size_t)kForceWaves * kTileF32) * sizeof(float4);
    int next = 0;
#define TPM_LAUNCH(KK)                                                                         \
    if (class_counts[KK - 1]) {                                                                \
        const uint32_t *starts = cls + kClsStarts + (KK - 1) * (kXcds + 1);                    \
        uint32_t *queue = cls + kClsQueue + (KK - 1) * kXcds;                                  \
        const uint32_t waves = class_counts[KK - 1];                                           \
        const uint32_t cap = (uint32_t)n_cu * (uint32_t)force_waves_per_simd(KK);              \
        const uint32_t want = (waves + kForceWaves - 1) / kForceWaves;                         \
        const uint32_t blocks = want < cap ? want : cap;                                       \
        hipStream_t s = streams[next++ % n_streams];                                           \
        if (rec64)                                                                             \
            k_force_f32<KK, 1><<<blocks, 64 * kForceWaves, lds, s>>>(                          \
                nd, gr, cls, starts, queue, off, len, entries, ps, pidx, fp, ft, rec);         \
        else                                                                                   \
            k_force_f32<KK, 0><<<blocks, 64 * kForceWaves, lds, s>>>(                          \
                nd, gr, cls, starts, queue, off, len, entries, ps, pidx, fp, ft, rec);         \
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

void launch_force_f32_multi(const ForceBox *boxes, int nb, const uint32_t *class_totals,
                            uint32_t max_entries, int n_cu, const hipStream_t *streams,
                            int n_streams)
{
    const size_t lds = ((size_t)max_entries + (size_t)kForceWaves * kTileF32) * sizeof(float4);
    int next = 0;
#define TPM_LAUNCH(KK)                                                                         \
    if (class_totals[KK - 1]) {                                                                \
        const uint32_t waves = class_totals[KK - 1];                                           \
        const uint32_t cap = (uint32_t)n_cu * (uint32_t)force_waves_per_simd(KK);              \
        const uint32_t want = (waves + kForceWaves - 1) / kForceWaves;                         \
        const uint32_t blocks = want < cap ? want : cap;                                       \
        k_force_f32_multi<KK><<<blocks, 64 * kForceWaves, lds,                                 \
                                streams[next++ % n_streams]>>>(boxes, nb);                     \
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

void launch_force_f32_prep(uint32_t *cls, hipStream_t s)
{
    fill_u32(cls + kClsQueue, kForceClasses * kXcds, 0u, s);
}

void launch_pairwise_f32(int64_t n_i, const double *xi, int64_t n_j, const double *xj,
                         const double *mj, const double *xg, double eta, ForceTable ft,
                         double *out, hipStream_t s)
{
    const double inv_len = 0.5 / eta; // 1 / r_cut
    const int64_t total = n_i * n_j;
    int64_t b = (total + 255) / 256;
    k_pairwise_f32<<<(unsigned)(b < 65536 ? (b > 0 ? b : 1) : 65536), 256, 0, s>>>(
        n_i, xi, n_j, xj, mj, xg[0], xg[1], xg[2], inv_len, ft, inv_len * inv_len, out);
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
                      ForceParams fp, void *rec, int rec64, hipStream_t s)
{
    if (!n_groups) return;
    if (rec64)
        k_force_f64<1><<<n_groups, 64, 0, s>>>(nd, gr, n_groups, off, len, entries, ps, pidx,
                                              fp, rec);
    else
        k_force_f64<0><<<n_groups, 64, 0, s>>>(nd, gr, n_groups, off, len, entries, ps, pidx,
                                              fp, rec);
}

void launch_force_out(const void *rec, int mode, int64_t n, void *ax, void *ay, void *az,
                      double dt, hipStream_t s)
{
    if (n <= 0) return;
    const int64_t want = (n + 255) / 256;
    const unsigned b = (unsigned)(want < 4096 ? want : 4096);
    if (mode == kOutKick)
        k_force_out<kOutKick><<<b, 256, 0, s>>>(rec, n, ax, ay, az, dt);
    else if (mode == kOutF64)
        k_force_out<kOutF64><<<b, 256, 0, s>>>(rec, n, ax, ay, az, dt);
    else
        k_force_out<kOutF32><<<b, 256, 0, s>>>(rec, n, ax, ay, az, dt);
}

// ------------------------------------------------------------------ the pair-law table
namespace {

// H(s) = g(R) / ((s + e2)^(3/2) (1 - s)^4), R = 2 sqrt(s) < 2 (lengths in units of r_cut), in
// double precision.  On eq. (2)'s first branch g is evaluated in the form without
// cancellation the FP64 kernel uses; on the second, g = (2 - R)^5 (7R^3 + 22R^2 + 10R + 4) / 140
// and 1 - s = (2 - R)(2 + R) / 4, so four of the five powers of (2 - R) cancel exactly.
double h_host(double s, double e2)
{
    const double R = 2.0 * std::sqrt(s), uncut = std::pow(s + e2, -1.5);
    if (R < 1.0) {
        const double R2 = R * R;
        const double g =
            1.0 + R2 * R * (-1.6 + R2 * (1.6 + R * (-0.5 + R * (-12.0 / 35.0 + 0.15 * R))));
        return g * uncut / std::pow(1.0 - s, 4);
    }
    return 256.0 * (2.0 - R) * (((7.0 * R + 22.0) * R + 10.0) * R + 4.0) /
           (140.0 * std::pow(2.0 + R, 4)) * uncut;
}

// Solves the 4 x 4 system M x = r (symmetric positive definite) by Gaussian elimination with
// partial pivoting.
void solve4(double M[4][4], double r[4], double x[4])
{
    for (int c = 0; c < 4; ++c) {
        int piv = c;
        for (int i = c + 1; i < 4; ++i)
            if (std::fabs(M[i][c]) > std::fabs(M[piv][c])) piv = i;
        for (int j = 0; j < 4; ++j) std::swap(M[c][j], M[piv][j]);
        std::swap(r[c], r[piv]);
        for (int i = c + 1; i < 4; ++i) {
            const double f = M[i][c] / M[c][c];
            for (int j = c; j < 4; ++j) M[i][j] -= f * M[c][j];
            r[i] -= f * r[c];
        }
    }
    for (int c = 3; c >= 0; --c) {
        double v = r[c];
        for (int j = c + 1; j < 4; ++j) v -= M[c][j] * x[j];
        x[c] = v / M[c][c];
    }
}

} // namespace

bool build_force_table(double eps_over_rcut, std::vector<float4> &coef, uint32_t &base, float &c)
{
    const double e2 = eps_over_rcut * eps_over_rcut;
    if (!(e2 > 0.0) || !std::isfinite(e2)) return false;
    // c: a power of two at most e2 / 64, so the pieces near s = 0 are narrow next to eps^2
    const int kc = (int)std::floor(std::log2(e2)) - 6;
    const int n_oct = -kc; // u in [2^kc, 1)
    const uint32_t pieces = (uint32_t)n_oct << kTabSegBits;
    if (n_oct < 1 || pieces + 1 > kTabMaxEntries) return false;
    const double cd = std::ldexp(1.0, kc);
    c = (float)cd;
    base = (uint32_t)(127 + kc) << kTabSegBits;
    coef.assign(pieces + 1, make_float4(0.f, 0.f, 0.f, 0.f));
    // Each piece: the cubic in x in [1, 2) (the position inside the piece, as the kernel forms
    // it) closest, in the relative least-squares sense at 16 Chebyshev nodes, to
    // H(s) = G(s) / (1 - s)^4.  H is smooth and positive below s = 1 (eq. 2's second branch
    // is (2 - R)^5 times a polynomial, and 1 - s = (2 - R)(2 + R) / 4), with a simple zero at
    // s = 1.
    constexpr int kNodes = 16;
    const double pi = 3.14159265358979323846;
    const double w_piece = 1.0 / (1 << kTabSegBits);
    for (uint32_t k = 0; k < pieces; ++k) {
        const int e = kc + (int)(k >> kTabSegBits);
        const double lo = std::ldexp(1.0 + (double)(k & ((1u << kTabSegBits) - 1)) * w_piece, e);
        const double w = std::ldexp(w_piece, e);
        double M[4][4] = {}, r[4] = {}, x[4];
        for (int i = 0; i < kNodes; ++i) {
            const double t = 0.5 * std::cos(pi * (i + 0.5) / kNodes); // in (-1/2, 1/2)
            const double s = lo + (t + 0.5) * w - cd;
            const double y = h_host(s, e2);
            const double wt = 1.0 / (y * y);
            const double x = t + 1.5;
            const double v[4] = {1.0, x, x * x, x * x * x};
            for (int a = 0; a < 4; ++a) {
                r[a] += wt * v[a] * y;
                for (int b = 0; b < 4; ++b) M[a][b] += wt * v[a] * v[b];
            }
        }
        solve4(M, r, x);
        coef[k] = make_float4((float)x[0], (float)x[1], (float)x[2], (float)x[3]);
    }
    return true;
}

} // namespace tpm
