// Barnes' group walk (Section 2.2 step 5): one shared interaction list per group.
//
// One 64-lane wavefront walks one group.  A stack of node indices lives in LDS; each step
// pops up to 64 nodes (one per lane), tests them in parallel and uses wave prefix sums to
// place the entries they emit and the children they push.  A step pops only as many nodes as
// leave kStackReserve slots free after their pushes (each pushes at most 8); when not even
// one fits, it pops one node, which continues the walk depth first: from a node at level l
// that needs at most 7 more slots per level below l, so the stack never outgrows kStackCap
// (wide walks, such as theta = 0, slow down instead of failing).  For each node, in FP64 and
// without FMA contraction (so the decisions equal a plain IEEE evaluation bit for bit):
//
//   prune  (beyond the cutoff from the group's box, cf. Section 2.2 step 3):
//          gap_a = max(0, |wrap(cn_a - cg_a)| - (l/2 + hg_a)),  gap^2 >= r_cut^2
//   accept (opening criterion measured from the box surface):
//          dc_a = max(0, |wrap(com_a - cg_a)| - hg_a),  l^2 < theta^2 dc^2  and gap^2 > 0
//          theta is fixed, or (distance-dependent opening, Section 4.1 eq. 12) the angle
//          theta(d) = min(theta_max, theta_0 / sqrt(R g(R))), R = d / eta, d = |dc|, taken
//          as theta_max where R g(R) = 0
//   leaf   : one particle entry per particle
//   else   : push the children.
//
// A list entry is a node index with kCellTag set (the node's mass at its centre of mass) or
// a particle's position in key order.  Group g's list is entries[off[g] .. off[g] + len[g]).
// Two ways to lay the lists out:
//   * two passes: the count pass records each group's list length; after a prefix sum the
//     emit pass writes the lists back to back.  The traversal order depends only on the tree,
//     so both passes visit the same nodes in the same order.
//   * one pass: a fixed set of waves takes groups in small batches from per-XCD counters;
//     each wave writes its lists back to back into chunks it takes from a shared pool with
//     one atomic per chunk (a list that does not fit the rest of a chunk is walked again into
//     a fresh one).  Pool and chunk sizes come from the caller (from an earlier walk); if a
//     list or the pool runs out of room, the pass reports it and the caller falls back to
//     two passes, so the result never depends on those sizes.
// Both layouts also run over the groups of several boxes in one launch (k_walk_multi,
// k_walk_pool_multi: per-box descriptors in device memory, each box's own lists and flags).
#include "common.hpp"

namespace tpm {
namespace {

constexpr int kStackCap = 1024;
constexpr int kStackReserve = 7 * kMaxLevel; // a depth-first descent from the root's children
constexpr uint32_t kWalkBatch = 4;

// |wrap(v)| for |v| <= L (both points in [0, L)): min(|v|, L - |v|).  Bit for bit the
// absolute value of the two-sided wrap (v - L if v >= L/2, v + L if v < -L/2, else v):
// the rounded L - |v| is the rounded |v -+ L|, and at |v| = L/2 both forms give L/2.
__device__ __forceinline__ double awrap(double v, double L)
{
    const double a = fabs(v);
    return fmin(a, L - a);
}

// Wave-wide prefix sums with DPP: four row shifts make inclusive sums inside each row of 16
// lanes, then two row broadcasts carry the row totals into the later rows.  The total is
// read from lane 63 into a scalar register, so values derived from it stay wave-uniform.
// Called with all 64 lanes active.
__device__ __forceinline__ uint32_t wave_excl_scan(uint32_t v, uint32_t *total)
{
    uint32_t x = v;
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xf, 0xf, true); // row_shr:1
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xf, 0xf, true); // row_shr:2
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xf, 0xf, true); // row_shr:4
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xf, 0xf, true); // row_shr:8
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xa, 0xf, false); // row_bcast:15
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xc, 0xf, false); // row_bcast:31
    *total = (uint32_t)__builtin_amdgcn_readlane((int)x, 63);
    return x - v;
}

// Wave-wide inclusive running maximum of a non-negative value (same DPP pattern as above;
// lanes shifted in from outside a row read 0, the identity here).
__device__ __forceinline__ uint32_t wave_incl_max(uint32_t x)
{
    x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xf, 0xf, true));
    x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xf, 0xf, true));
    x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xf, 0xf, true));
    x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xf, 0xf, true));
    x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xa, 0xf, false));
    x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xc, 0xf, false));
    return x;
}

// g_P3M(R) of eq. (2) in its expanded polynomial form, evaluated term by term from the
// powers R^2 .. R^8 so that the opening decisions it feeds are plain IEEE FP64 operations.
__device__ __forceinline__ double g_p3m_expanded(double R)
{
    const double R2 = R * R, R3 = R2 * R, R4 = R3 * R, R5 = R4 * R, R6 = R5 * R, R7 = R6 * R,
                 R8 = R7 * R;
    if (R < 1.0)
        return 1.0 - (224.0 * R3 - 224.0 * R5 + 70.0 * R6 + 48.0 * R7 - 21.0 * R8) / 140.0;
    if (R < 2.0)
        return 1.0 - (12.0 - 224.0 * R2 + 896.0 * R3 - 840.0 * R4 + 224.0 * R5 + 70.0 * R6 -
                      48.0 * R7 + 7.0 * R8) / 140.0;
    return 0.0;
}

// theta(d) of eq. (12) with the distance in units of eta and the cap theta_max.  sqrt and
// the divisions are the correctly rounded FP64 operations.
__device__ __forceinline__ double theta_of_d(double d, const WalkParams &wp)
{
    const double R = d / wp.eta;
    const double s = R * g_p3m_expanded(R);
    if (!(s > 0.0)) return wp.theta_max;
    const double th = wp.theta0 / sqrt(s);
    return th < wp.theta_max ? th : wp.theta_max;
}

struct Visit {
    int kind; // 0 skip, 1 cell entry, 2 leaf particles, 3 open
    uint32_t ne, np, f, cf;
};

// The decision for a node with record w (see the top of this file).  OPEN: 0 fixed theta,
// 1 distance-dependent theta(d).
template <int OPEN>
__device__ __forceinline__ Visit visit(const WalkNode &w, const WalkParams &wp, double cg0,
                                       double cg1, double cg2, double hg0, double hg1,
                                       double hg2)
{
    Visit r{0, 0u, 0u, 0u, 0u};
    const double L = wp.L;
    const double l = ldexp(L, -(int)w.level); // L / 2^level, exact
    const double half = l * 0.5;
    double v0 = awrap(w.cn[0] - cg0, L) - (half + hg0);
    double v1 = awrap(w.cn[1] - cg1, L) - (half + hg1);
    double v2 = awrap(w.cn[2] - cg2, L) - (half + hg2);
    double gp0 = v0 > 0.0 ? v0 : 0.0, gp1 = v1 > 0.0 ? v1 : 0.0, gp2 = v2 > 0.0 ? v2 : 0.0;
    double G = gp0 * gp0 + gp1 * gp1 + gp2 * gp2;
    if (G < wp.rc2) {
        double w0 = awrap(w.com[0] - cg0, L) - hg0;
        double w1 = awrap(w.com[1] - cg1, L) - hg1;
        double w2 = awrap(w.com[2] - cg2, L) - hg2;
        double d0 = w0 > 0.0 ? w0 : 0.0, d1 = w1 > 0.0 ? w1 : 0.0, d2 = w2 > 0.0 ? w2 : 0.0;
        const double D = d0 * d0 + d1 * d1 + d2 * d2;
        const double ll = l * l;
        bool take = ll < wp.th2 * D;
        if (OPEN && take && !(ll < wp.th2lo * D)) {
            // theta_lo <= theta(d) <= theta_max, and rounding is monotone, so only nodes in
            // the band between the two bounds need the angle itself.
            const double th = theta_of_d(sqrt(D), wp);
            take = ll < (th * th) * D;
        }
        if (take && G > 0.0) {
            r.kind = 1;
            r.ne = 1;
        } else if (w.nchild == 0) {
            r.kind = 2;
            r.f = w.first;
            r.ne = w.count;
        } else {
            r.kind = 3;
            r.cf = w.child_first;
            r.np = w.nchild;
        }
    }
    return r;
}

// How many nodes a step pops from a stack holding `top`: at most 64, and only as many as leave
// kStackReserve slots free after their pushes (each pushes at most 8), but at least one.
__device__ __forceinline__ int pop_count(int top)
{
    int room = (kStackCap - kStackReserve - top) / 7;
    int k = top < 64 ? top : 64;
    if (room < 1) room = 1;
    return k > room ? room : k;
}

// The node a lane pops (lanes at or past k read the root, node 0, and ignore it).
__device__ __forceinline__ uint32_t pop_node(const uint32_t *stk, int top, int k, int lane,
                                             const WalkParams &wp, unsigned *overflow)
{
    uint32_t u = lane < k ? stk[top - k + lane] : 0u;
    if (u >= wp.n_nodes) { // cannot happen for a well-formed tree: report, never read
        atomicOr(overflow, 2u);
        u = 0u;
    }
    return u;
}

// Walks group g with the calling wave.  EMIT: writes the list to dst[0 .. cap) (entries past
// cap are counted but not stored).  Returns the list length; *ncell gets the cell entries.
// stk (kStackCap) and s_mark (64) are the wave's LDS scratch.  Each step visits the popped
// nodes, pushes the children of the opened ones, pops the next step's nodes and starts
// reading their records, and only then writes this step's list entries, so the writes
// overlap the reads.
template <int EMIT, int OPEN>
__device__ __forceinline__ uint64_t walk_group(const WalkNode *__restrict__ wn,
                                               const GroupArrays &gr, uint32_t g,
                                               const WalkParams &wp, uint32_t *stk,
                                               uint32_t *s_mark, uint32_t *__restrict__ dst,
                                               uint64_t cap, unsigned *overflow,
                                               uint64_t *ncell_out)
{
    const int lane = threadIdx.x;
    const double cg0 = gr.cgx[g], cg1 = gr.cgy[g], cg2 = gr.cgz[g];
    const double hg0 = gr.hgx[g], hg1 = gr.hgy[g], hg2 = gr.hgz[g];
    uint64_t written = 0, ncell = 0;
    // the first step pops the root alone
    int k = 1, top = 0;
    uint32_t u = 0u;
    WalkNode rec = wn[0];
    while (k > 0) {
        Visit a{0, 0u, 0u, 0u, 0u};
        if (lane < k) a = visit<OPEN>(rec, wp, cg0, cg1, cg2, hg0, hg1, hg2);
        uint32_t ne_tot, np_tot;
        const uint32_t ne_ex = wave_excl_scan(a.ne, &ne_tot);
        const uint32_t np_ex = wave_excl_scan(a.np, &np_tot);
        if (top + (int)np_tot > kStackCap) {
            if (lane == 0) atomicOr(overflow, 1u);
            break;
        }
        __syncthreads(); // the last step's stack reads are done before these pushes
        if (a.kind == 3)
            for (uint32_t c = 0; c < a.np; ++c) stk[top + np_ex + c] = a.cf + c;
        top += (int)np_tot;
        __syncthreads(); // pushes visible before the pops
        const int k2 = top > 0 ? pop_count(top) : 0;
        const uint32_t u2 = pop_node(stk, top, k2, lane, wp, overflow);
        const WalkNode rec2 = wn[u2];
        top -= k2;
        if (EMIT && ne_tot) {
            // Expand this step's entries cooperatively so the global writes are contiguous,
            // 64 slots at a time.  Each lane whose run starts inside the chunk marks its
            // start slot with lane + 1; a running maximum over the chunk's slots then names
            // the owner of every slot (the previous chunk's last owner carries over).
            uint32_t carry = 0;
            const uint32_t val = a.kind == 1 ? (u | kCellTag) : a.f;
            for (uint32_t base = 0; base < ne_tot; base += 64) {
                s_mark[lane] = 0u;
                __syncthreads();
                if (a.ne && ne_ex >= base && ne_ex < base + 64) s_mark[ne_ex - base] = lane + 1;
                __syncthreads();
                uint32_t own = wave_incl_max(s_mark[lane]);
                own = max(own, carry);
                carry = (uint32_t)__builtin_amdgcn_readlane((int)own, 63);
                const int src = (int)own - 1;
                const uint32_t v = (uint32_t)__shfl((int)val, src, 64);
                const uint32_t ex = (uint32_t)__shfl((int)ne_ex, src, 64);
                const int cell = __shfl(a.kind == 1 ? 1 : 0, src, 64);
                const uint32_t q = base + lane;
                if (q < ne_tot && written + q < cap) dst[written + q] = cell ? v : v + (q - ex);
            }
        }
        written += ne_tot;
        ncell += (uint64_t)__popcll(__ballot(a.kind == 1));
        k = k2;
        u = u2;
        rec = rec2;
    }
    __syncthreads(); // the stack and marks are free for the next group
    *ncell_out = ncell;
    return written;
}

// Two passes, one wave per group.  Count: cnt[g] = list length.  Emit: writes the list at
// entries + off[g], and len[g], gcells[g].
template <int EMIT, int OPEN>
__global__ __launch_bounds__(64) void k_walk(const WalkNode *__restrict__ wn, GroupArrays gr,
                                             uint32_t n_groups, WalkParams wp,
                                             uint64_t *__restrict__ cnt_off,
                                             uint32_t *__restrict__ len,
                                             uint32_t *__restrict__ entries,
                                             unsigned *overflow, uint32_t *__restrict__ gcells)
{
    __shared__ uint32_t stk[kStackCap];
    __shared__ uint32_t s_mark[64];
    const uint32_t g = xcd_block(blockIdx.x, gridDim.x);
    if (g >= n_groups) return;
    uint64_t ncell = 0;
    const uint64_t w = walk_group<EMIT, OPEN>(wn, gr, g, wp, stk, s_mark,
                                        EMIT ? entries + cnt_off[g] : nullptr, ~0ull, overflow,
                                        &ncell);
    if (threadIdx.x == 0) {
        if (!EMIT) {
            cnt_off[g] = w;
        } else {
            len[g] = (uint32_t)w;
            gcells[g] = (uint32_t)ncell;
        }
    }
}

// One pass: groups are split into kXcds equal ranges with a counter each; a wave takes
// kWalkBatch groups at a time from its own range (b mod kXcds, the XCD the block is dealt
// to), then from the others, so every wave ends once all counters have passed their ranges.
// Lists go into chunks of `chunk` entries taken from the pool (entries[0, pool_cap)) through
// *pool_next.  A group is walked into the current chunk if at least `reserve` entries are
// left there; if its list did not fit (or there was no such room) the wave takes a fresh
// chunk and walks the group into that.  A list longer than a chunk, or an exhausted pool,
// sets bit 4 of *overflow and ends the wave.
template <int OPEN>
__global__ __launch_bounds__(64) void k_walk_pool(const WalkNode *__restrict__ wn,
                                                  GroupArrays gr, uint32_t n_groups,
                                                  WalkParams wp, uint32_t *counters,
                                                  unsigned long long *pool_next,
                                                  uint64_t pool_cap, uint64_t chunk,
                                                  uint64_t reserve, uint64_t *__restrict__ off,
                                                  uint32_t *__restrict__ len,
                                                  uint32_t *__restrict__ entries,
                                                  unsigned *overflow,
                                                  uint32_t *__restrict__ gcells)
{
    __shared__ uint32_t stk[kStackCap];
    __shared__ uint32_t s_mark[64];
    uint64_t cur = 0, end = 0; // the wave's current chunk [cur, end)
    const uint32_t x0 = blockIdx.x % kXcds;
    for (uint32_t r = 0; r < kXcds; ++r) {
        const uint32_t x = (x0 + r) % kXcds;
        const uint32_t lo = (uint32_t)((uint64_t)n_groups * x / kXcds);
        const uint32_t hi = (uint32_t)((uint64_t)n_groups * (x + 1) / kXcds);
        for (;;) {
            uint32_t t = 0;
            if (threadIdx.x == 0) t = atomicAdd(&counters[x], kWalkBatch);
            t = (uint32_t)__builtin_amdgcn_readfirstlane((int)t);
            if (t >= hi - lo) break;
            const uint32_t g1 = lo + t + kWalkBatch < hi ? lo + t + kWalkBatch : hi;
            for (uint32_t g = lo + t; g < g1; ++g) {
                uint64_t ncell = 0, w = 0;
                bool fits = false;
                if (end - cur >= reserve) { // room for a list of typical length: try here
                    w = walk_group<1, OPEN>(wn, gr, g, wp, stk, s_mark, entries + cur, end - cur,
                                      overflow, &ncell);
                    fits = w <= end - cur;
                }
                if (!fits) { // a fresh chunk, and the walk again if it had not fitted
                    unsigned long long c0 = 0;
                    if (threadIdx.x == 0) c0 = atomicAdd(pool_next, (unsigned long long)chunk);
                    const uint32_t c_lo =
                        (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)c0);
                    const uint32_t c_hi =
                        (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(c0 >> 32));
                    cur = ((uint64_t)c_hi << 32) | c_lo;
                    end = cur + chunk;
                    if (end > pool_cap) {
                        if (threadIdx.x == 0) atomicOr(overflow, 4u);
                        return;
                    }
                    w = walk_group<1, OPEN>(wn, gr, g, wp, stk, s_mark, entries + cur, chunk,
                                      overflow, &ncell);
                    if (w > chunk) {
                        if (threadIdx.x == 0) atomicOr(overflow, 4u);
                        return;
                    }
                }
                if (threadIdx.x == 0) {
                    off[g] = cur;
                    len[g] = (uint32_t)w;
                    gcells[g] = (uint32_t)ncell;
                }
                cur += w;
            }
        }
    }
}

// ------------------------------------------------------------------ several boxes at once
// The box of work item t: the last box whose first item is at most t (uniform reads).
__device__ __forceinline__ int box_of(const WalkBox *__restrict__ bx, int nb, uint32_t t)
{
    int b = 0;
    while (b + 1 < nb && bx[b + 1].g0 <= t) ++b;
    return b;
}

// Group g of box B with that box's opening rule.
template <int EMIT>
__device__ __forceinline__ uint64_t walk_box_group(const WalkBox &B, uint32_t g, uint32_t *stk,
                                                   uint32_t *s_mark, uint32_t *dst, uint64_t cap,
                                                   uint64_t *ncell)
{
    if (B.wp.open)
        return walk_group<EMIT, 1>(B.wn, B.gr, g, B.wp, stk, s_mark, dst, cap, B.overflow,
                                   ncell);
    return walk_group<EMIT, 0>(B.wn, B.gr, g, B.wp, stk, s_mark, dst, cap, B.overflow, ncell);
}

// The two passes of k_walk over the items of several boxes, one wave per item.
template <int EMIT>
__global__ __launch_bounds__(64) void k_walk_multi(const WalkBox *__restrict__ bx, int nb,
                                                   uint32_t total)
{
    __shared__ uint32_t stk[kStackCap];
    __shared__ uint32_t s_mark[64];
    const uint32_t t = xcd_block(blockIdx.x, gridDim.x);
    if (t >= total) return;
    const WalkBox &B = bx[box_of(bx, nb, t)];
    const uint32_t g = t - B.g0;
    uint64_t ncell = 0;
    const uint64_t w =
        walk_box_group<EMIT>(B, g, stk, s_mark, EMIT ? B.entries + B.off[g] : nullptr, ~0ull,
                             &ncell);
    if (threadIdx.x == 0) {
        if (!EMIT) {
            B.off[g] = w;
        } else {
            B.len[g] = (uint32_t)w;
            B.gcells[g] = (uint32_t)ncell;
        }
    }
}

// k_walk_pool over the items of several boxes.  A wave's chunk belongs to one box: at the
// first item of another box it takes a fresh chunk from that box's pool.  A list that does
// not fit a chunk, or an exhausted pool, flags its box (bit 4) and the wave goes on with the
// next item, so the other boxes' lists are complete.
__global__ __launch_bounds__(64) void k_walk_pool_multi(const WalkBox *__restrict__ bx, int nb,
                                                        uint32_t total, uint32_t *counters)
{
    __shared__ uint32_t stk[kStackCap];
    __shared__ uint32_t s_mark[64];
    uint64_t cur = 0, end = 0; // the wave's current chunk [cur, end) of box cb
    int cb = -1;
    const uint32_t x0 = blockIdx.x % kXcds;
    for (uint32_t r = 0; r < kXcds; ++r) {
        const uint32_t x = (x0 + r) % kXcds;
        const uint32_t lo = (uint32_t)((uint64_t)total * x / kXcds);
        const uint32_t hi = (uint32_t)((uint64_t)total * (x + 1) / kXcds);
        for (;;) {
            uint32_t k = 0;
            if (threadIdx.x == 0) k = atomicAdd(&counters[x], kWalkBatch);
            k = (uint32_t)__builtin_amdgcn_readfirstlane((int)k);
            if (k >= hi - lo) break;
            const uint32_t t1 = lo + k + kWalkBatch < hi ? lo + k + kWalkBatch : hi;
            for (uint32_t t = lo + k; t < t1; ++t) {
                const int b = box_of(bx, nb, t);
                const WalkBox &B = bx[b];
                if (b != cb) {
                    cb = b;
                    cur = end = 0;
                }
                const uint32_t g = t - B.g0;
                uint64_t ncell = 0, w = 0;
                bool fits = false;
                if (end - cur >= B.reserve) {
                    w = walk_box_group<1>(B, g, stk, s_mark, B.entries + cur, end - cur, &ncell);
                    fits = w <= end - cur;
                }
                if (!fits) {
                    unsigned long long c0 = 0;
                    if (threadIdx.x == 0) c0 = atomicAdd(B.pool_next, (unsigned long long)B.chunk);
                    const uint32_t c_lo =
                        (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)c0);
                    const uint32_t c_hi =
                        (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(c0 >> 32));
                    cur = ((uint64_t)c_hi << 32) | c_lo;
                    end = cur + B.chunk;
                    if (end > B.pool_cap) {
                        if (threadIdx.x == 0) atomicOr(B.overflow, 4u);
                        cur = end = 0;
                        continue;
                    }
                    w = walk_box_group<1>(B, g, stk, s_mark, B.entries + cur, B.chunk, &ncell);
                    if (w > B.chunk) {
                        if (threadIdx.x == 0) atomicOr(B.overflow, 4u);
                        cur = end = 0;
                        continue;
                    }
                }
                if (threadIdx.x == 0) {
                    B.off[g] = cur;
                    B.len[g] = (uint32_t)w;
                    B.gcells[g] = (uint32_t)ncell;
                }
                cur += w;
            }
        }
    }
}

// (cell entries, particle entries, interactions = sum_g count_g * L_g): block reductions and
// one atomic per block.
__global__ __launch_bounds__(256) void k_walk_stats(GroupArrays gr, uint32_t n_groups,
                                                    const uint32_t *__restrict__ len,
                                                    const uint32_t *__restrict__ gcells,
                                                    unsigned long long *stats)
{
    unsigned long long c = 0, p = 0, it = 0, mx = 0;
    for (uint32_t g = blockIdx.x * blockDim.x + threadIdx.x; g < n_groups;
         g += gridDim.x * blockDim.x) {
        const unsigned long long l = len[g];
        c += gcells[g];
        p += l - gcells[g];
        it += l * gr.count[g];
        mx = l > mx ? l : mx;
    }
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) {
        const unsigned long long o = __shfl_xor(mx, d, 64);
        mx = o > mx ? o : mx;
    }
    if ((threadIdx.x & 63) == 0) atomicMax(&stats[3], mx);
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) {
        c += __shfl_xor(c, d, 64);
        p += __shfl_xor(p, d, 64);
        it += __shfl_xor(it, d, 64);
    }
    __shared__ unsigned long long sm[3][4];
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        sm[0][w] = c;
        sm[1][w] = p;
        sm[2][w] = it;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        unsigned long long t = sm[threadIdx.x][0] + sm[threadIdx.x][1] + sm[threadIdx.x][2] +
                               sm[threadIdx.x][3];
        atomicAdd(&stats[threadIdx.x], t);
    }
}

} // namespace

void launch_walk_count(const WalkNode *wn, GroupArrays gr, uint32_t n_groups, WalkParams wp,
                       uint64_t *counts, unsigned *overflow, hipStream_t s)
{
    if (!n_groups) return;
    if (wp.open)
        k_walk<0, 1><<<n_groups, 64, 0, s>>>(wn, gr, n_groups, wp, counts, nullptr, nullptr,
                                            overflow, nullptr);
    else
        k_walk<0, 0><<<n_groups, 64, 0, s>>>(wn, gr, n_groups, wp, counts, nullptr, nullptr,
                                            overflow, nullptr);
}

void launch_walk_emit(const WalkNode *wn, GroupArrays gr, uint32_t n_groups, WalkParams wp,
                      const uint64_t *off, uint32_t *len, uint32_t *entries, unsigned *overflow,
                      uint32_t *gcells, hipStream_t s)
{
    if (!n_groups) return;
    if (wp.open)
        k_walk<1, 1><<<n_groups, 64, 0, s>>>(wn, gr, n_groups, wp, const_cast<uint64_t *>(off),
                                            len, entries, overflow, gcells);
    else
        k_walk<1, 0><<<n_groups, 64, 0, s>>>(wn, gr, n_groups, wp, const_cast<uint64_t *>(off),
                                            len, entries, overflow, gcells);
}

void launch_walk_pool(const WalkNode *wn, GroupArrays gr, uint32_t n_groups, WalkParams wp,
                      uint32_t n_waves, uint64_t pool_cap, uint64_t chunk, uint64_t reserve,
                      uint32_t *counters, uint64_t *off, uint32_t *len, uint32_t *entries,
                      unsigned *overflow, uint32_t *gcells, hipStream_t s)
{
    if (!n_groups) return;
    fill_u32(counters, kXcds + 2, 0u, s);
    if (wp.open)
        k_walk_pool<1><<<n_waves, 64, 0, s>>>(wn, gr, n_groups, wp, counters,
                                              (unsigned long long *)(counters + kXcds),
                                              pool_cap, chunk, reserve, off, len, entries,
                                              overflow, gcells);
    else
        k_walk_pool<0><<<n_waves, 64, 0, s>>>(wn, gr, n_groups, wp, counters,
                                              (unsigned long long *)(counters + kXcds),
                                              pool_cap, chunk, reserve, off, len, entries,
                                              overflow, gcells);
}

void launch_walk_count_multi(const WalkBox *boxes, int nb, uint32_t total, hipStream_t s)
{
    if (total) k_walk_multi<0><<<total, 64, 0, s>>>(boxes, nb, total);
}

void launch_walk_emit_multi(const WalkBox *boxes, int nb, uint32_t total, hipStream_t s)
{
    if (total) k_walk_multi<1><<<total, 64, 0, s>>>(boxes, nb, total);
}

void launch_walk_pool_multi(const WalkBox *boxes, int nb, uint32_t total, uint32_t n_waves,
                            uint32_t *counters, hipStream_t s)
{
    if (!total) return;
    fill_u32(counters, kXcds, 0u, s);
    k_walk_pool_multi<<<n_waves, 64, 0, s>>>(boxes, nb, total, counters);
}

void launch_walk_stats(GroupArrays gr, uint32_t n_groups, const uint32_t *len,
                       const uint32_t *gcells, unsigned long long *stats, hipStream_t s)
{
    if (!n_groups) return;
    unsigned b = (n_groups + 255) / 256;
    k_walk_stats<<<b < 256 ? b : 256, 256, 0, s>>>(gr, n_groups, len, gcells, stats);
}

} // namespace tpm
