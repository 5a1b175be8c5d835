// Tree construction kernels (Section 2.2 step 2): input validation and 63-bit Morton keys,
// stable LSD radix sort of (key, index), gather into key order, the octree built level by
// level with the N_leaf stopping rule (Section 3.1.2), FP64 node masses and centres of mass,
// and the N_crit groups of Barnes' interaction-list method.
//
// Every floating-point operation here is FP64 and this file is compiled without FMA
// contraction: keys, node moments, group boxes and cube centres must equal, bit for bit,
// what a plain IEEE evaluation of the same expressions gives, so that the walk takes exactly
// the decisions the definition takes.
#include "common.hpp"

namespace tpm {
namespace {

__device__ __forceinline__ uint64_t spread3(uint64_t v)
{
    v &= 0x1fffffull;
    v = (v | v << 32) & 0x1f00000000ffffull;
    v = (v | v << 16) & 0x1f0000ff0000ffull;
    v = (v | v << 8) & 0x100f00f00f00f00full;
    v = (v | v << 4) & 0x10c30c30c30c30c3ull;
    v = (v | v << 2) & 0x1249249249249249ull;
    return v;
}

__device__ __forceinline__ uint32_t compact3(uint64_t v)
{
    v &= 0x1249249249249249ull;
    v = (v ^ (v >> 2)) & 0x10c30c30c30c30c3ull;
    v = (v ^ (v >> 4)) & 0x100f00f00f00f00full;
    v = (v ^ (v >> 8)) & 0x1f0000ff0000ffull;
    v = (v ^ (v >> 16)) & 0x1f00000000ffffull;
    v = (v ^ (v >> 32)) & 0x1fffffull;
    return (uint32_t)v;
}

// q = min(2^21 - 1, floor(p * 2^21 / L)), clamped at 0 for safety (validated separately).
__device__ __forceinline__ uint64_t quantise(double p, double scale)
{
    double f = floor(p * scale);
    if (!(f > 0.0)) return 0;
    if (f >= 2097151.0) return 2097151ull;
    return (uint64_t)f;
}

__global__ __launch_bounds__(256) void k_keys(int64_t n, const double *__restrict__ x,
                                              const double *__restrict__ y,
                                              const double *__restrict__ z,
                                              const double *__restrict__ m, double L,
                                              double scale, uint64_t *__restrict__ key,
                                              uint32_t *__restrict__ idx, unsigned *flags,
                                              double4 *__restrict__ rec)
{
    unsigned f = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        double p0 = x[i], p1 = y[i], p2 = z[i], mi = m[i];
        if (!isfinite(p0) || !isfinite(p1) || !isfinite(p2) || !isfinite(mi) || !(mi > 0.0))
            f |= kFlagNonFinite;
        else if (!(p0 >= 0.0 && p0 < L && p1 >= 0.0 && p1 < L && p2 >= 0.0 && p2 < L))
            f |= kFlagRange;
        uint64_t k = (spread3(quantise(p0, scale)) << 2) | (spread3(quantise(p1, scale)) << 1) |
                     spread3(quantise(p2, scale));
        key[i] = k;
        idx[i] = (uint32_t)i;
        rec[i] = make_double4(p0, p1, p2, mi);
    }
    if (f) atomicOr(flags, f);
}

__global__ __launch_bounds__(kSortThreads) void k_hist(const uint64_t *__restrict__ key,
                                                       int64_t n, int shift,
                                                       uint32_t *__restrict__ hist,
                                                       uint32_t nblocks)
{
    __shared__ uint32_t h[kSortBins];
    h[threadIdx.x] = 0;
    __syncthreads();
    int64_t base = (int64_t)blockIdx.x * kSortTile;
    for (int it = 0; it < kSortItems; ++it) {
        int64_t k = base + (int64_t)it * kSortThreads + threadIdx.x;
        if (k < n) atomicAdd(&h[(uint32_t)(key[k] >> shift) & (kSortBins - 1)], 1u);
    }
    __syncthreads();
    hist[(size_t)threadIdx.x * nblocks + blockIdx.x] = h[threadIdx.x];
}

// Stable scatter of one tile.  Wave w takes elements w * 1024 + it * 64 + lane of the tile
// (iteration it = 0..15), which is also their order for stability.  Each wave ranks its
// elements among equal digits with ballots and a wave-private running count per digit (no
// block barrier inside the loop); the per-wave counts then give each wave's base inside
// each digit's run.  The tile is reordered by digit in LDS and written out in that order,
// so elements with equal digits leave as contiguous runs.
__global__ __launch_bounds__(kSortThreads) void k_scatter(const uint64_t *__restrict__ key,
                                                          const uint32_t *__restrict__ idx,
                                                          int64_t n, int shift,
                                                          const uint32_t *__restrict__ hist,
                                                          uint32_t nblocks,
                                                          uint64_t *__restrict__ key_out,
                                                          uint32_t *__restrict__ idx_out)
{
    constexpr int kWaves = kSortThreads / 64;
    __shared__ uint64_t skey[kSortTile];
    __shared__ uint32_t sidx[kSortTile];
    __shared__ uint32_t goff[kSortBins];  // global offset of this tile's digit-d run
    __shared__ uint32_t loff[kSortBins];  // local offset of digit d inside the tile
    __shared__ uint32_t wcnt[kWaves][kSortBins]; // per-wave digit counts, then wave bases
    __shared__ uint32_t wsum[kWaves];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
    goff[tid] = hist[(size_t)tid * nblocks + blockIdx.x];
#pragma unroll
    for (int q = 0; q < kWaves; ++q) wcnt[q][tid] = 0;
    __syncthreads();
    const uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;
    const int64_t wb = base + (int64_t)w * (kSortItems * 64);
    uint64_t kv[kSortItems];
    uint32_t iv[kSortItems], rk[kSortItems];
#pragma unroll
    for (int it = 0; it < kSortItems; ++it) {
        const int64_t k = wb + it * 64 + lane;
        const bool valid = k < n;
        kv[it] = valid ? key[k] : 0ull;
        iv[it] = valid ? idx[k] : 0u;
    }
#pragma unroll
    for (int it = 0; it < kSortItems; ++it) {
        const bool valid = wb + it * 64 + lane < n;
        const uint32_t d = (uint32_t)(kv[it] >> shift) & (kSortBins - 1);
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < kSortBits; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t bb = __ballot(bit);
            peers &= bit ? bb : ~bb;
        }
        // LDS operations of one wave complete in order: every lane reads the running
        // count before the lowest lane of each digit advances it.
        const uint32_t before = valid ? wcnt[w][d] : 0u;
        rk[it] = before + (uint32_t)__popcll(peers & lt);
        if (valid && (peers & lt) == 0) wcnt[w][d] = before + (uint32_t)__popcll(peers);
    }
    __syncthreads();
    {
        // digit tid: wave bases inside its run, then the exclusive scan over digits
        uint32_t v = 0;
#pragma unroll
        for (int q = 0; q < kWaves; ++q) {
            const uint32_t c = wcnt[q][tid];
            wcnt[q][tid] = v;
            v += c;
        }
        uint32_t inc = v;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const uint32_t o = __shfl_up(inc, d, 64);
            if (lane >= d) inc += o;
        }
        if (lane == 63) wsum[w] = inc;
        __syncthreads();
        uint32_t before = 0;
        for (int q = 0; q < w; ++q) before += wsum[q];
        loff[tid] = before + inc - v;
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < kSortItems; ++it) {
        if (wb + it * 64 + lane < n) {
            const uint32_t d = (uint32_t)(kv[it] >> shift) & (kSortBins - 1);
            const uint32_t lp = loff[d] + wcnt[w][d] + rk[it];
            skey[lp] = kv[it];
            sidx[lp] = iv[it];
        }
    }
    __syncthreads();
    const int64_t cnt = (n - base) < kSortTile ? (n - base) : kSortTile;
    for (int e = tid; e < cnt; e += kSortThreads) {
        const uint64_t kk = skey[e];
        const uint32_t d = (uint32_t)(kk >> shift) & (kSortBins - 1);
        const uint32_t pos = goff[d] + ((uint32_t)e - loff[d]);
        key_out[pos] = kk;
        idx_out[pos] = sidx[e];
    }
}

// Second half of the sort.  After stable passes over the key bits from kRunBits up, equal
// high parts form runs (cells of about level 13, rarely more than a few particles) in input
// order; sorting each run by (key, index) completes the order by (key, index).  One thread
// per run start sorts a run of up to kShortRun elements in registers; longer runs, up to
// kLongRun, are listed for k_fix_long_runs; a run longer than that (or a full list) sets
// *fallback, and the caller then sorts everything by all bits.  Elements of one run share the
// high part, so reading neighbours while their runs are being reordered is harmless.
__global__ __launch_bounds__(256) void k_fix_runs(int64_t n, uint64_t *__restrict__ key,
                                                  uint32_t *__restrict__ idx,
                                                  uint2 *__restrict__ long_runs,
                                                  uint32_t long_cap, unsigned *long_count,
                                                  unsigned *fallback)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t hk = key[i] >> kRunBits;
        if (i > 0 && (key[i - 1] >> kRunBits) == hk) continue;
        int64_t e = i + 1;
        while (e < n && e - i <= (int64_t)kLongRun && (key[e] >> kRunBits) == hk) ++e;
        const int64_t len = e - i;
        if (len > (int64_t)kShortRun) {
            const unsigned slot = len <= (int64_t)kLongRun ? atomicAdd(long_count, 1u) : long_cap;
            if (slot < long_cap)
                long_runs[slot] = make_uint2((uint32_t)i, (uint32_t)len);
            else
                atomicOr(fallback, 1u);
            continue;
        }
        if (len == 1) continue;
        // up to kShortRun (8) elements: Batcher's odd-even merge network in registers, the
        // unused slots padded with keys above every real one
        uint64_t k8[8];
        uint32_t v8[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            k8[q] = ~0ull;
            v8[q] = ~0u;
            if (q < len) {
                k8[q] = key[i + q];
                v8[q] = idx[i + q];
            }
        }
        constexpr int8_t net[19][2] = {{0, 1}, {2, 3}, {4, 5}, {6, 7}, {0, 2}, {1, 3}, {4, 6},
                                       {5, 7}, {1, 2}, {5, 6}, {0, 4}, {1, 5}, {2, 6}, {3, 7},
                                       {2, 4}, {3, 5}, {1, 2}, {3, 4}, {5, 6}};
#pragma unroll
        for (int c = 0; c < 19; ++c) {
            const int a = net[c][0], b = net[c][1];
            const bool swap = k8[a] > k8[b] || (k8[a] == k8[b] && v8[a] > v8[b]);
            const uint64_t ka = swap ? k8[b] : k8[a], kb = swap ? k8[a] : k8[b];
            const uint32_t va = swap ? v8[b] : v8[a], vb = swap ? v8[a] : v8[b];
            k8[a] = ka;
            k8[b] = kb;
            v8[a] = va;
            v8[b] = vb;
        }
#pragma unroll
        for (int q = 0; q < 8; ++q)
            if (q < len) {
                key[i + q] = k8[q];
                idx[i + q] = v8[q];
            }
    }
}

// Listed runs, one block each: the run is staged in LDS and every element is written to the
// position given by its rank, the number of elements before it in (key, index) order.
__global__ __launch_bounds__(256) void k_fix_long_runs(const uint2 *__restrict__ long_runs,
                                                       const unsigned *long_count,
                                                       uint32_t long_cap,
                                                       uint64_t *__restrict__ key,
                                                       uint32_t *__restrict__ idx)
{
    __shared__ uint64_t sk[kLongRun];
    __shared__ uint32_t si[kLongRun];
    unsigned cnt = *long_count;
    cnt = cnt < long_cap ? cnt : long_cap;
    for (unsigned r = blockIdx.x; r < cnt; r += gridDim.x) {
        const uint2 run = long_runs[r];
        const uint32_t f = run.x, len = run.y;
        for (uint32_t j = threadIdx.x; j < len; j += blockDim.x) {
            sk[j] = key[f + j];
            si[j] = idx[f + j];
        }
        __syncthreads();
        for (uint32_t j = threadIdx.x; j < len; j += blockDim.x) {
            const uint64_t kj = sk[j];
            const uint32_t vj = si[j];
            uint32_t rank = 0;
            for (uint32_t q = 0; q < len; ++q)
                rank += (sk[q] < kj || (sk[q] == kj && si[q] < vj)) ? 1u : 0u;
            key[f + rank] = kj;
            idx[f + rank] = vj;
        }
        __syncthreads();
    }
}

// Gather the (x, y, z, m) records into key order.
// Records in key order, and the largest mass (its bit pattern: masses are positive, so the
// patterns order like the values) into *mmax, which the caller has zeroed.  A block adds its
// maximum only when it exceeds the value already there, so equal masses cost one atomic.
__global__ __launch_bounds__(256) void k_permute(int64_t n, const uint32_t *__restrict__ idx,
                                                 const double4 *__restrict__ rec,
                                                 double4 *__restrict__ psrc,
                                                 unsigned long long *mmax)
{
    unsigned long long v = 0;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n;
         k += (int64_t)gridDim.x * blockDim.x) {
        const double4 r = rec[idx[k]];
        psrc[k] = r;
        const unsigned long long b = (unsigned long long)__double_as_longlong(r.w);
        v = b > v ? b : v;
    }
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) {
        const unsigned long long o = __shfl_xor(v, d, 64);
        v = o > v ? o : v;
    }
    __shared__ unsigned long long wm[4];
    if ((threadIdx.x & 63) == 0) wm[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < 4; ++w) v = wm[w] > v ? wm[w] : v;
        if (v > *(volatile unsigned long long *)mmax) atomicMax(mmax, v);
    }
}

// Cube centre of a node from its code: ((i + 0.5) * L / 2^level) per axis.
__device__ __forceinline__ void cube_centre(uint64_t code, int level, double L, double *c)
{
    uint64_t pre = code ^ (1ull << (3 * level));
    double l = ldexp(L, -level);
    c[0] = ((double)compact3(pre >> 2) + 0.5) * l;
    c[1] = ((double)compact3(pre >> 1) + 0.5) * l;
    c[2] = ((double)compact3(pre) + 0.5) * l;
}

__global__ void k_root(NodeArrays nd, uint32_t n, double L)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        nd.code[0] = 1;
        nd.first[0] = 0;
        nd.count[0] = n;
        nd.parent[0] = 0;
        nd.level[0] = 0;
        nd.nchild[0] = 0;
        nd.child_first[0] = 0;
        double c[3];
        cube_centre(1, 0, L, c);
        nd.cnx[0] = c[0];
        nd.cny[0] = c[1];
        nd.cnz[0] = c[2];
    }
}

// Boundaries of the 8 octants of a node's key range at the next level: b[o] = first sorted
// position whose next-level digit is >= o; b[8] = end.
__device__ __forceinline__ void octant_bounds(const uint64_t *__restrict__ key, uint32_t f,
                                              uint32_t c, int level, uint32_t *b)
{
    int shift = 3 * (kMaxLevel - (level + 1));
    b[0] = f;
    b[8] = f + c;
    for (int o = 1; o < 8; ++o) {
        uint32_t lo = b[o - 1], hi = f + c;
        while (lo < hi) {
            uint32_t mid = lo + ((hi - lo) >> 1);
            if ((int)((key[mid] >> shift) & 7u) < o)
                lo = mid + 1;
            else
                hi = mid;
        }
        b[o] = lo;
    }
}

// Octant bounds of subdivided nodes are stored per level, seven per node (b[1..7]; b[0] and
// b[8] are the node's first and end), by k_split or k_split_wide and read back by k_emit.
__global__ __launch_bounds__(256) void k_split(NodeArrays nd, const uint64_t *__restrict__ key,
                                               uint32_t lo, uint32_t hi, int level, int n_leaf,
                                               uint32_t *__restrict__ cnt,
                                               uint32_t *__restrict__ bnd)
{
    for (uint32_t u = lo + blockIdx.x * blockDim.x + threadIdx.x; u < hi;
         u += gridDim.x * blockDim.x) {
        uint32_t c = nd.count[u];
        uint32_t nch = 0;
        if ((int64_t)c >= n_leaf && level < kMaxLevel) {
            uint32_t b[9];
            octant_bounds(key, nd.first[u], c, level, b);
            for (int o = 0; o < 8; ++o) nch += (b[o + 1] > b[o]);
            uint32_t *q = bnd + (size_t)(u - lo) * 7;
            for (int o = 1; o < 8; ++o) q[o - 1] = b[o];
        }
        nd.nchild[u] = (uint8_t)nch;
        cnt[u - lo] = nch;
    }
}

// The same for levels of few, large nodes: one wave per node, each octant boundary found by
// a 64-way search (each round samples 64 keys of the current interval and keeps the gap
// where the digit reaches the octant), so a node of c particles takes about log64(c) rounds
// of one parallel load instead of log2(c) dependent loads.
__global__ __launch_bounds__(256) void k_split_wide(NodeArrays nd,
                                                    const uint64_t *__restrict__ key,
                                                    uint32_t lo, uint32_t hi, int level,
                                                    int n_leaf, uint32_t *__restrict__ cnt,
                                                    uint32_t *__restrict__ bnd)
{
    const uint32_t u = lo + blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const uint32_t lane = threadIdx.x & 63;
    if (u >= hi) return; // the whole wave leaves together
    const uint32_t f = nd.first[u], c = nd.count[u];
    uint32_t nch = 0;
    if ((int64_t)c >= n_leaf && level < kMaxLevel) {
        const int shift = 3 * (kMaxLevel - (level + 1));
        uint32_t prev = f;
        nch = 0;
        for (uint32_t o = 1; o <= 8; ++o) {
            uint32_t bo = f + c;
            if (o < 8) {
                // first position in [prev, f + c) whose digit is >= o; it lies in [l, h]
                uint32_t l = prev, h = f + c;
                while (h - l > 64) {
                    const uint32_t sj = l + (uint32_t)((uint64_t)(h - l) * (lane + 1) / 65);
                    const bool below = (uint32_t)((key[sj] >> shift) & 7u) < o;
                    const uint32_t t = (uint32_t)__popcll(__ballot(below));
                    const uint32_t s_lo = l + (uint32_t)((uint64_t)(h - l) * t / 65);
                    const uint32_t s_hi = l + (uint32_t)((uint64_t)(h - l) * (t + 1) / 65);
                    // samples 0..t-1 are below o, sample t (if any) is not
                    if (t > 0) l = s_lo + 1;
                    if (t < 64) h = s_hi;
                }
                const uint32_t p = l + lane;
                const bool below = p < h && (uint32_t)((key[p] >> shift) & 7u) < o;
                bo = l + (uint32_t)__popcll(__ballot(below));
                if (lane == 0) bnd[(size_t)(u - lo) * 7 + (o - 1)] = bo;
            }
            nch += (bo > prev);
            prev = bo;
        }
    }
    if (lane == 0) {
        nd.nchild[u] = (uint8_t)nch;
        cnt[u - lo] = nch;
    }
}

__global__ __launch_bounds__(256) void k_emit(NodeArrays nd, const uint32_t *__restrict__ bnd,
                                              uint32_t lo, uint32_t hi, int level,
                                              uint32_t base, const uint32_t *__restrict__ cnt,
                                              double L)
{
    for (uint32_t u = lo + blockIdx.x * blockDim.x + threadIdx.x; u < hi;
         u += gridDim.x * blockDim.x) {
        uint32_t nch = nd.nchild[u];
        if (!nch) {
            nd.child_first[u] = 0;
            continue;
        }
        uint32_t cf = base + cnt[u - lo];
        nd.child_first[u] = cf;
        uint32_t b[9];
        b[0] = nd.first[u];
        b[8] = b[0] + nd.count[u];
        const uint32_t *q = bnd + (size_t)(u - lo) * 7;
        for (int o = 1; o < 8; ++o) b[o] = q[o - 1];
        uint64_t pc = nd.code[u];
        uint32_t v = cf;
        for (int o = 0; o < 8; ++o) {
            if (b[o + 1] <= b[o]) continue;
            uint64_t code = (pc << 3) | (uint64_t)o;
            nd.code[v] = code;
            nd.first[v] = b[o];
            nd.count[v] = b[o + 1] - b[o];
            nd.parent[v] = u;
            nd.level[v] = (uint8_t)(level + 1);
            nd.nchild[v] = 0;
            double cc[3];
            cube_centre(code, level + 1, L, cc);
            nd.cnx[v] = cc[0];
            nd.cny[v] = cc[1];
            nd.cnz[v] = cc[2];
            ++v;
        }
    }
}

// ---------------------------------------------------------------- octree from the sorted keys
// The tree of the level-by-level split, built in three passes without per-level searches.
// With d_i the number of levels (leading key digits) particle i shares with particle i - 1,
// particle i is the first particle of one cell at every level from s_i = d_i + 1 on (s_0 = 0:
// the root).  A cell at level l >= 1 is a node iff its parent cell holds at least n_leaf
// particles and l <= 21; counts only shrink down the tree, so the parent's ancestors are then
// subdivided too.  The parent of particle i's level-l cell holds at least n_leaf particles iff
// some n_leaf consecutive particles including i share l - 1 levels; so with m_a the levels
// particles a and a + n_leaf - 1 share, lambda_i = max of m_a over the windows
// a = i - n_leaf + 1 .. i, i's leaf is at level L_i = min(lambda_i + 1, 21) (L_i = 0 if the box
// holds fewer than n_leaf particles), and the nodes that start at particle i are its cells at
// levels s_i .. L_i.  Stored level by level and within a level by first particle (the order
// the level-by-level split produces), node (l, i) has index off[l] + (level-l nodes that start
// before i); its first child, if any, is node (l + 1, i); its parent is the last level-(l - 1)
// node that starts at or before i.
constexpr int kTreeThreads = 256;
constexpr int kTreeItems = 16;
constexpr int kTreeTile = kTreeThreads * kTreeItems;
constexpr int kTreeLevels = kMaxLevel + 1;
constexpr uint32_t kTreeLong = 0x3fffffu; // leaf count not found within the window

// This wave's LDS writes are complete before any of its lanes reads LDS again.
__device__ __forceinline__ void wave_sync_lds()
{
    __builtin_amdgcn_s_waitcnt(0xc07f); // lgkmcnt(0); vector memory counters untouched
    __builtin_amdgcn_wave_barrier();
}

// Levels two keys share: 21 if equal, else the number of equal leading 3-bit digits.
__device__ __forceinline__ int shared_levels(uint64_t a, uint64_t b)
{
    const uint64_t x = a ^ b;
    if (!x) return kMaxLevel;
    const int h = 63 - (int)__clzll((long long)x);
    return kMaxLevel - 1 - h / 3;
}

// Per particle i a packed word: s_i (bits 0-4; 22 if no node starts there), L_i (bits 5-9)
// and, if a node starts at i, the particle count of its leaf (L_i, i) (bits 10-31; kTreeLong if
// that leaf is a level-21 cell longer than the window, found later by a search).  Per block,
// the number of nodes of each level that start in its tile: blk[l * nblk + b].  The block
// keeps in LDS, as bytes, the levels shared by each window and the first level of a cell at
// each particle, over [b0 - W, b0 + tile + W), W = n_leaf - 1: the window maxima need W
// windows before the tile, and a leaf below level 21 holds fewer than n_leaf particles, so its
// end lies within W particles after its first.
__device__ __forceinline__ uint32_t tree_word(int s, int Lf, uint32_t cnt)
{
    return (uint32_t)s | ((uint32_t)Lf << 5) | (cnt << 10);
}

__global__ __launch_bounds__(kTreeThreads) void k_tree_levels(const uint64_t *__restrict__ key,
                                                             uint32_t n, int n_leaf,
                                                             uint32_t *__restrict__ sl,
                                                             uint32_t *__restrict__ blk,
                                                             uint32_t nblk)
{
    __shared__ uint8_t ms[kTreeTile + kTreeWin];
    __shared__ uint8_t ss[kTreeTile + kTreeWin];
    __shared__ uint32_t lc[kTreeLevels];
    const uint32_t b = blockIdx.x;
    const int W = n_leaf - 1;
    const int64_t b0 = (int64_t)b * kTreeTile, k0 = b0 - W;
    if (threadIdx.x < kTreeLevels) lc[threadIdx.x] = 0u;
    // ms[t]: levels shared by the window a = k0 + t (its first and last particle), 0xff if
    // there is no such window (a < 0 or a + W >= n); ss[t]: s of particle j = b0 + t, the
    // first level of a cell starting there (0 for the first particle; 0xff past the end)
    const int64_t last_a = (int64_t)n - n_leaf;
    for (int t = threadIdx.x; t < kTreeTile + W; t += kTreeThreads) {
        const int64_t a = k0 + t;
        ms[t] = (a >= 0 && a <= last_a) ? (uint8_t)shared_levels(key[a], key[a + W])
                                        : (uint8_t)0xff;
        const int64_t j = b0 + t;
        ss[t] = j >= (int64_t)n ? (uint8_t)0xff
                : j == 0        ? (uint8_t)0
                                : (uint8_t)(shared_levels(key[j - 1], key[j]) + 1);
    }
    __syncthreads();
    // item q of thread x is particle b0 + q * kTreeThreads + x (neighbouring lanes read
    // neighbouring LDS bytes); lm[q]: the levels s .. L of the nodes that start there
    uint32_t lm[kTreeItems];
#pragma unroll
    for (int q = 0; q < kTreeItems; ++q) {
        const int tt = q * kTreeThreads + (int)threadIdx.x; // particle b0 + tt
        const int64_t i = b0 + tt;
        lm[q] = 0u;
        if (i >= (int64_t)n) continue;
        const int t = tt + W; // position of window i in ms
        const int s = ss[tt];
        int lam = -1;
        for (int a = t - W; a <= t; ++a) {
            const int m = ms[a];
            if (m != 0xff && m > lam) lam = m;
        }
        const int Lf = (int64_t)n < n_leaf ? 0 : min(lam + 1, kMaxLevel);
        uint32_t cnt = 0;
        if (s <= Lf) {
            // the leaf (Lf, i) ends at the first j > i where a cell of level <= Lf starts
            // (ss = 0xff past the last particle ends it too); below level 21 it holds at
            // most W particles, so the end lies within W
            cnt = kTreeLong;
            for (int d = 1; d <= W; ++d) {
                if (ss[tt + d] <= Lf || ss[tt + d] == 0xff) {
                    cnt = (uint32_t)d;
                    break;
                }
            }
            lm[q] = (2u << Lf) - (1u << s);
        }
        sl[i] = tree_word(s <= Lf ? s : 22, Lf, cnt);
    }
    // nodes per level starting in this tile: one ballot per level and item, one LDS add per
    // level and wave
#pragma unroll
    for (int l = 0; l < kTreeLevels; ++l) {
        uint32_t c = 0;
#pragma unroll
        for (int q = 0; q < kTreeItems; ++q) c += (uint32_t)__popcll(__ballot((lm[q] >> l) & 1u));
        if ((threadIdx.x & 63) == 0 && c) atomicAdd(&lc[l], c);
    }
    __syncthreads();
    if (threadIdx.x < kTreeLevels) blk[(size_t)threadIdx.x * nblk + b] = lc[threadIdx.x];
}

// One block per level: exclusive prefix over the blocks' counts, in place; the level's total
// into tot[l].
__global__ __launch_bounds__(1024) void k_tree_scan(uint32_t *__restrict__ blk, uint32_t nblk,
                                                    uint32_t *__restrict__ tot)
{
    __shared__ uint32_t part[1024];
    uint32_t *row = blk + (size_t)blockIdx.x * nblk;
    const uint32_t per = (nblk + 1023) / 1024;
    const uint32_t lo = min(threadIdx.x * per, nblk), hi = min(lo + per, nblk);
    uint32_t sum = 0;
    for (uint32_t j = lo; j < hi; ++j) sum += row[j];
    part[threadIdx.x] = sum;
    __syncthreads();
    for (int d = 1; d < 1024; d <<= 1) {
        const uint32_t v = (int)threadIdx.x >= d ? part[threadIdx.x - d] : 0u;
        __syncthreads();
        part[threadIdx.x] += v;
        __syncthreads();
    }
    uint32_t run = threadIdx.x ? part[threadIdx.x - 1] : 0u;
    for (uint32_t j = lo; j < hi; ++j) {
        const uint32_t v = row[j];
        row[j] = run;
        run += v;
    }
    if (threadIdx.x == 1023) tot[blockIdx.x] = part[1023];
}

// First particle after i outside the cell that holds i at the level of shift sh (p = key[i]
// >> sh): a doubling search, then bisection.
__device__ __forceinline__ uint32_t cell_end(const uint64_t *__restrict__ key, uint32_t n,
                                             uint32_t i, int sh, uint64_t p)
{
    uint64_t lo = i, hi = n, step = 1;
    for (;;) {
        const uint64_t j = lo + step;
        if (j >= n) break;
        if ((key[j] >> sh) != p) {
            hi = j;
            break;
        }
        lo = j;
        step <<= 1;
    }
    while (hi - lo > 1) { // key[lo] is in the cell, hi is not (or n)
        const uint64_t mid = lo + ((hi - lo) >> 1);
        if ((key[mid] >> sh) == p)
            lo = mid;
        else
            hi = mid;
    }
    return (uint32_t)hi;
}

// Every node, at its index: code, first, level, parent, cube centre, child_first = the index
// its first child has or would have (the moments pass derives nchild from it), and the count
// of leaves (internal counts are summed by the moments pass).  Level by level, each wave lists
// the particles of its tile part at which a node of that level starts (in particle order, so
// in node order) and then writes 64 consecutive nodes at a time.  msk[l][t]: which of thread
// t's 16 particles start a level-l node; cur[l][t]: the index of the first of them.
__global__ __launch_bounds__(kTreeThreads) void k_tree_emit(NodeArrays nd,
                                                           const uint64_t *__restrict__ key,
                                                           const uint32_t *__restrict__ sl,
                                                           const uint32_t *__restrict__ blk,
                                                           uint32_t nblk, TreeOffsets to,
                                                           uint32_t n, double L)
{
    __shared__ uint32_t cur[kTreeLevels][kTreeThreads];
    __shared__ uint16_t msk[kTreeLevels][kTreeThreads];
    __shared__ uint16_t lst[kTreeThreads / 64][64 * kTreeItems];
    const uint32_t b = blockIdx.x, tid = threadIdx.x;
    const int64_t b0 = (int64_t)b * kTreeTile;
    const int64_t i0 = b0 + (int64_t)tid * kTreeItems;
    uint32_t w[kTreeItems];
#pragma unroll
    for (int q = 0; q < kTreeItems; ++q) {
        const int64_t i = i0 + q;
        w[q] = i < (int64_t)n ? sl[i] : 22u; // s = 22: no node
    }
    for (int l = 0; l < kTreeLevels; ++l) {
        uint32_t m = 0;
#pragma unroll
        for (int q = 0; q < kTreeItems; ++q) {
            const int s = (int)(w[q] & 31u), Lf = (int)((w[q] >> 5) & 31u);
            m |= (s <= l && l <= Lf) ? (1u << q) : 0u;
        }
        msk[l][tid] = (uint16_t)m;
        cur[l][tid] = (uint32_t)__popc(m);
    }
    __syncthreads();
    // each level's counts, exclusive prefix over the threads (wave v takes levels v, v + 4,
    // ...; a lane holds four threads' counts), plus the level offset and the block's base
    const int wave = tid >> 6, lane = tid & 63;
    for (int l = wave; l < kTreeLevels; l += kTreeThreads / 64) {
        const uint32_t x0 = cur[l][4 * lane], x1 = cur[l][4 * lane + 1],
                       x2 = cur[l][4 * lane + 2], x3 = cur[l][4 * lane + 3];
        const uint32_t s4 = x0 + x1 + x2 + x3;
        uint32_t incl = s4;
        for (int d = 1; d < 64; d <<= 1) {
            const uint32_t y = (uint32_t)__shfl_up((int)incl, d, 64);
            if (lane >= d) incl += y;
        }
        uint32_t ex = incl - s4 + blk[(size_t)l * nblk + b] + to.off[l];
        cur[l][4 * lane] = ex;
        ex += x0;
        cur[l][4 * lane + 1] = ex;
        ex += x1;
        cur[l][4 * lane + 2] = ex;
        ex += x2;
        cur[l][4 * lane + 3] = ex;
    }
    __syncthreads();
    uint16_t *my = lst[wave];
    const uint32_t t0 = (uint32_t)wave * 64; // first thread of this wave
    for (int l = 0; l < kTreeLevels; ++l) {
        const uint32_t base = cur[l][t0];
        const uint32_t total = cur[l][t0 + 63] + (uint32_t)__popc(msk[l][t0 + 63]) - base;
        if (!total) continue; // the same on every lane
        // list this lane's particles in node order
        uint32_t m = msk[l][tid], pos = cur[l][tid] - base;
        while (m) {
            const int q = __ffs((int)m) - 1;
            m &= m - 1u;
            my[pos++] = (uint16_t)(tid * kTreeItems + q);
        }
        wave_sync_lds();
        const int sh = 3 * (kMaxLevel - l);
        for (uint32_t j = lane; j < total; j += 64) {
            const uint32_t p = my[j];
            const uint32_t t = p >> 4, q = p & 15u;
            const uint32_t i = (uint32_t)b0 + p;
            const uint32_t u = base + j;
            const uint64_t k = key[i];
            const uint64_t code = (k >> sh) | (1ull << (3 * l));
            nd.code[u] = code;
            nd.first[u] = i;
            nd.level[u] = (uint8_t)l;
            nd.nchild[u] = 0;
            nd.parent[u] =
                l ? cur[l - 1][t] + (uint32_t)__popc(msk[l - 1][t] & ((2u << q) - 1u)) - 1u : 0u;
            nd.child_first[u] =
                l < kMaxLevel ? cur[l + 1][t] + (uint32_t)__popc(msk[l + 1][t] & ((1u << q) - 1u))
                              : to.off[kTreeLevels];
            const uint32_t wi = sl[i];
            uint32_t cnt = 0;
            if ((int)((wi >> 5) & 31u) == l) {
                cnt = wi >> 10;
                if (cnt == kTreeLong) cnt = cell_end(key, n, i, sh, k >> sh) - i;
            }
            nd.count[u] = cnt;
            double cc[3];
            cube_centre(code, l, L, cc);
            nd.cnx[u] = cc[0];
            nd.cny[u] = cc[1];
            nd.cnz[u] = cc[2];
        }
        wave_sync_lds(); // the list is read before the next level rewrites it
    }
}

// Moments of the nodes [lo, hi) of one level, from their particles (leaves) or their children
// in octant order: mass and mass-weighted position sums S (kept for the parents), and the
// node's final records, the source (S / M, M) and the walk record.  DERIVE (a tree from
// k_tree_emit): a node's children are the next level's nodes from its child_first up to the
// child_first of the next node of its level (child_end after the level's last node), so
// nchild is set here, and an internal node's count is the sum of its children's.
template <int DERIVE>
__global__ __launch_bounds__(256) void k_moments(NodeArrays nd, const double4 *__restrict__ ps,
                                                 uint32_t lo, uint32_t hi, uint32_t child_end,
                                                 WalkNode *__restrict__ wn)
{
    for (uint32_t u = lo + blockIdx.x * blockDim.x + threadIdx.x; u < hi;
         u += gridDim.x * blockDim.x) {
        double M = 0.0, Sx = 0.0, Sy = 0.0, Sz = 0.0;
        uint32_t nch;
        if (DERIVE) {
            const uint32_t nx = u + 1 < hi ? nd.child_first[u + 1] : child_end;
            nch = nx - nd.child_first[u];
            nd.nchild[u] = (uint8_t)nch;
        } else {
            nch = nd.nchild[u];
        }
        const uint32_t f = nd.first[u];
        uint32_t cnt, cf = 0;
        if (nch == 0) {
            cnt = nd.count[u];
            for (uint32_t k = f; k < f + cnt; ++k) {
                const double4 r = ps[k];
                M += r.w;
                Sx += r.w * r.x;
                Sy += r.w * r.y;
                Sz += r.w * r.z;
            }
        } else {
            cf = nd.child_first[u];
            cnt = 0;
            for (uint32_t c = cf; c < cf + nch; ++c) {
                M += nd.mass[c];
                Sx += nd.comx[c];
                Sy += nd.comy[c];
                Sz += nd.comz[c];
                cnt += nd.count[c];
            }
            if (DERIVE) nd.count[u] = cnt;
        }
        nd.mass[u] = M;
        nd.comx[u] = Sx;
        nd.comy[u] = Sy;
        nd.comz[u] = Sz;
        const double c0 = Sx / M, c1 = Sy / M, c2 = Sz / M;
        nd.nsrc[u] = make_double4(c0, c1, c2, M);
        WalkNode w;
        w.cn[0] = nd.cnx[u];
        w.cn[1] = nd.cny[u];
        w.cn[2] = nd.cnz[u];
        w.com[0] = c0;
        w.com[1] = c1;
        w.com[2] = c2;
        w.first = f;
        w.count = cnt;
        w.nchild = (uint8_t)nch;
        w.child_first = cf;
        w.level = nd.level[u];
        w.pad0 = w.pad1 = 0;
        wn[u] = w;
    }
}

__global__ __launch_bounds__(256) void k_group_mark(NodeArrays nd, uint32_t n_nodes, int n_crit,
                                                    uint32_t *__restrict__ gstart,
                                                    uint32_t *__restrict__ gflag)
{
    for (uint32_t u = blockIdx.x * blockDim.x + threadIdx.x; u < n_nodes;
         u += gridDim.x * blockDim.x) {
        int64_t c = nd.count[u];
        bool cand = (c <= n_crit) || nd.nchild[u] == 0;
        bool top = (u == 0) || ((int64_t)nd.count[nd.parent[u]] > n_crit);
        if (cand && top) {
            uint32_t f = nd.first[u];
            gstart[f] = u + 1;
            gflag[f] = 1;
        }
    }
}

__global__ __launch_bounds__(256) void k_group_compact(const uint32_t *__restrict__ gstart,
                                                       const uint32_t *__restrict__ gpos,
                                                       int64_t n, uint32_t *__restrict__ gnode)
{
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n;
         k += (int64_t)gridDim.x * blockDim.x) {
        uint32_t s = gstart[k];
        if (s) gnode[gpos[k]] = s - 1;
    }
}

// Eight lanes per group: exact min/max of its particle positions.
__global__ __launch_bounds__(256) void k_group_bbox(NodeArrays nd, GroupArrays gr,
                                                    uint32_t n_groups,
                                                    const double4 *__restrict__ ps)
{
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t g = t >> 3;
    const int sub = (int)(t & 7);
    const bool act = g < n_groups;
    uint32_t u = 0, f = 0, c = 0;
    if (act) {
        u = gr.node[g];
        f = nd.first[u];
        c = nd.count[u];
    }
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (uint32_t k = f + sub; k < f + c; k += 8) {
        const double4 r = ps[k];
        double p[3] = {r.x, r.y, r.z};
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            lo[a] = fmin(lo[a], p[a]);
            hi[a] = fmax(hi[a], p[a]);
        }
    }
    // the eight lanes of a group are an aligned run of the wave
#pragma unroll
    for (int d = 4; d > 0; d >>= 1) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            lo[a] = fmin(lo[a], __shfl_xor(lo[a], d, 64));
            hi[a] = fmax(hi[a], __shfl_xor(hi[a], d, 64));
        }
    }
    if (act && sub == 0) {
        gr.first[g] = f;
        gr.count[g] = c;
        gr.lox[g] = lo[0]; gr.loy[g] = lo[1]; gr.loz[g] = lo[2];
        gr.hix[g] = hi[0]; gr.hiy[g] = hi[1]; gr.hiz[g] = hi[2];
        gr.cgx[g] = (lo[0] + hi[0]) * 0.5;
        gr.cgy[g] = (lo[1] + hi[1]) * 0.5;
        gr.cgz[g] = (lo[2] + hi[2]) * 0.5;
        gr.hgx[g] = (hi[0] - lo[0]) * 0.5;
        gr.hgy[g] = (hi[1] - lo[1]) * 0.5;
        gr.hgz[g] = (hi[2] - lo[2]) * 0.5;
        gr.xgx[g] = nd.cnx[u];
        gr.xgy[g] = nd.cny[u];
        gr.xgz[g] = nd.cnz[u];
    }
}

// Shallowest group level and largest group: block reductions, one atomic per block.
__global__ __launch_bounds__(256) void k_group_extremes(NodeArrays nd, GroupArrays gr,
                                                        uint32_t n_groups, unsigned *min_level,
                                                        unsigned *max_count)
{
    unsigned lv = 255u, mc = 0u;
    for (uint32_t g = blockIdx.x * blockDim.x + threadIdx.x; g < n_groups;
         g += gridDim.x * blockDim.x) {
        uint32_t u = gr.node[g];
        lv = min(lv, (unsigned)nd.level[u]);
        mc = max(mc, (unsigned)nd.count[u]);
    }
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) {
        lv = min(lv, (unsigned)__shfl_xor((int)lv, d, 64));
        mc = max(mc, (unsigned)__shfl_xor((int)mc, d, 64));
    }
    __shared__ unsigned s_lv[4], s_mc[4];
    if ((threadIdx.x & 63) == 0) {
        s_lv[threadIdx.x >> 6] = lv;
        s_mc[threadIdx.x >> 6] = mc;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < 4; ++w) {
            lv = min(lv, s_lv[w]);
            mc = max(mc, s_mc[w]);
        }
        atomicMin(min_level, lv);
        atomicMax(max_count, mc);
    }
}

inline unsigned grid_for(int64_t n, int threads, int64_t cap = 65536)
{
    int64_t b = (n + threads - 1) / threads;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return (unsigned)b;
}

} // namespace

void launch_keys(int64_t n, const double *x, const double *y, const double *z, const double *m,
                 double L, uint64_t *key, uint32_t *idx, unsigned *flags, double4 *rec,
                 hipStream_t s)
{
    double scale = 2097152.0 / L;
    k_keys<<<grid_for(n, 256), 256, 0, s>>>(n, x, y, z, m, L, scale, key, idx, flags, rec);
}

size_t sort_hist_elems(int64_t n)
{
    size_t nb = (size_t)((n + kSortTile - 1) / kSortTile);
    if (nb < 1) nb = 1;
    return nb * kSortBins;
}

// Stable LSD passes over bits [lo_bit, 64) of the keys, 8 bits per pass; an even number of
// passes leaves the result in key / idx.
static void radix_passes(int64_t n, int lo_bit, uint64_t *key, uint32_t *idx, uint64_t *key_alt,
                         uint32_t *idx_alt, uint32_t *hist, uint32_t *scan_tmp, hipStream_t s)
{
    uint32_t nb = (uint32_t)((n + kSortTile - 1) / kSortTile);
    uint64_t *kin = key, *kout = key_alt;
    uint32_t *iin = idx, *iout = idx_alt;
    for (int shift = lo_bit; shift < 64; shift += kSortBits) {
        k_hist<<<nb, kSortThreads, 0, s>>>(kin, n, shift, hist, nb);
        scan_u32(hist, (size_t)nb * kSortBins, scan_tmp, scan_tmp + 1, s);
        k_scatter<<<nb, kSortThreads, 0, s>>>(kin, iin, n, shift, hist, nb, kout, iout);
        uint64_t *tk = kin; kin = kout; kout = tk;
        uint32_t *ti = iin; iin = iout; iout = ti;
    }
}

bool radix_sort_high(int64_t n, uint64_t *key, uint32_t *idx, uint64_t *key_alt,
                     uint32_t *idx_alt, uint32_t *hist, uint32_t *scan_tmp, uint2 *long_runs,
                     uint32_t long_cap, unsigned *flags, hipStream_t s)
{
    fill_u32(flags, 2, 0u, s); // [0] listed long runs, [1] fallback
    if (n <= 1) return false;
    radix_passes(n, kRunBits, key, idx, key_alt, idx_alt, hist, scan_tmp, s);
    const bool odd = ((64 - kRunBits) / kSortBits) % 2 == 1;
    uint64_t *k = odd ? key_alt : key;
    uint32_t *v = odd ? idx_alt : idx;
    k_fix_runs<<<grid_for(n, 256), 256, 0, s>>>(n, k, v, long_runs, long_cap, flags, flags + 1);
    k_fix_long_runs<<<256, 256, 0, s>>>(long_runs, flags, long_cap, k, v);
    return odd;
}

void radix_sort(int64_t n, uint64_t *key, uint32_t *idx, uint64_t *key_alt, uint32_t *idx_alt,
                uint32_t *hist, uint32_t *scan_tmp, hipStream_t s)
{
    if (n <= 1) return;
    radix_passes(n, 0, key, idx, key_alt, idx_alt, hist, scan_tmp, s);
}

void launch_permute(int64_t n, const uint32_t *idx, const double4 *rec, double4 *psrc,
                    unsigned long long *mmax, hipStream_t s)
{
    fill_u64((uint64_t *)mmax, 1, 0ull, s);
    if (n) k_permute<<<grid_for(n, 256), 256, 0, s>>>(n, idx, rec, psrc, mmax);
}

void launch_root(NodeArrays nd, uint32_t n, double L, hipStream_t s)
{
    k_root<<<1, 64, 0, s>>>(nd, n, L);
}

void launch_split(NodeArrays nd, const uint64_t *key, uint32_t lo, uint32_t hi, int level,
                  int n_leaf, uint32_t *cnt, uint32_t *bnd, hipStream_t s)
{
    if (hi - lo <= kWideSplitNodes)
        k_split_wide<<<(hi - lo + 3) / 4, 256, 0, s>>>(nd, key, lo, hi, level, n_leaf, cnt, bnd);
    else
        k_split<<<grid_for(hi - lo, 256), 256, 0, s>>>(nd, key, lo, hi, level, n_leaf, cnt, bnd);
}
void launch_emit(NodeArrays nd, const uint32_t *bnd, uint32_t lo, uint32_t hi, int level,
                 uint32_t base, const uint32_t *cnt, double L, hipStream_t s)
{
    k_emit<<<grid_for(hi - lo, 256), 256, 0, s>>>(nd, bnd, lo, hi, level, base, cnt, L);
}

void launch_moments(NodeArrays nd, const double4 *ps, uint32_t lo, uint32_t hi, int derive,
                    uint32_t child_end, WalkNode *wn, hipStream_t s)
{
    if (hi <= lo) return;
    if (derive)
        k_moments<1><<<grid_for(hi - lo, 256), 256, 0, s>>>(nd, ps, lo, hi, child_end, wn);
    else
        k_moments<0><<<grid_for(hi - lo, 256), 256, 0, s>>>(nd, ps, lo, hi, child_end, wn);
}

uint32_t tree_blocks(int64_t n) { return (uint32_t)((n + kTreeTile - 1) / kTreeTile); }

void launch_tree_levels(const uint64_t *key, uint32_t n, int n_leaf, uint32_t *sl, uint32_t *blk,
                        uint32_t *tot, hipStream_t s)
{
    const uint32_t nblk = tree_blocks(n);
    k_tree_levels<<<nblk, kTreeThreads, 0, s>>>(key, n, n_leaf, sl, blk, nblk);
    k_tree_scan<<<kTreeLevels, 1024, 0, s>>>(blk, nblk, tot);
}

void launch_tree_emit(NodeArrays nd, const uint64_t *key, const uint32_t *sl, const uint32_t *blk,
                      const TreeOffsets &to, uint32_t n, double L, hipStream_t s)
{
    const uint32_t nblk = tree_blocks(n);
    k_tree_emit<<<nblk, kTreeThreads, 0, s>>>(nd, key, sl, blk, nblk, to, n, L);
}


void launch_group_mark(NodeArrays nd, uint32_t n_nodes, int n_crit, uint32_t *gstart,
                       uint32_t *gflag, int64_t n, hipStream_t s)
{
    fill_u32(gstart, (size_t)n, 0u, s);
    fill_u32(gflag, (size_t)n + 1, 0u, s);
    k_group_mark<<<grid_for(n_nodes, 256), 256, 0, s>>>(nd, n_nodes, n_crit, gstart, gflag);
}

void launch_group_compact(const uint32_t *gstart, const uint32_t *gpos, int64_t n,
                          uint32_t *gnode, hipStream_t s)
{
    k_group_compact<<<grid_for(n, 256), 256, 0, s>>>(gstart, gpos, n, gnode);
}

void launch_group_bbox(NodeArrays nd, GroupArrays gr, uint32_t n_groups, const double4 *ps,
                       unsigned *min_level, unsigned *max_count, hipStream_t s)
{
    if (!n_groups) return;
    k_group_bbox<<<(unsigned)(((uint64_t)n_groups * 8 + 255) / 256), 256, 0, s>>>(nd, gr, n_groups,
                                                                                ps);
    k_group_extremes<<<grid_for(n_groups, 256, 256), 256, 0, s>>>(nd, gr, n_groups, min_level,
                                                                 max_count);
}

} // namespace tpm
