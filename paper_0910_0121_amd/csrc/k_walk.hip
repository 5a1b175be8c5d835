// Barnes' group walk (Section 2.2 step 5): one shared interaction list per group.
//
// One 64-lane wavefront walks one group.  A stack of node indices lives in LDS; each step
// pops up to 64 nodes (one per lane), tests them in parallel and uses wave prefix sums to
// place the entries they emit and the children they push.  For each node, in FP64 and
// without FMA contraction (so the decisions equal a plain IEEE evaluation bit for bit):
//
//   prune  (beyond the cutoff from the group's box, cf. Section 2.2 step 3):
//          gap_a = max(0, |wrap(cn_a - cg_a)| - (l/2 + hg_a)),  gap^2 >= r_cut^2
//   accept (opening criterion measured from the box surface):
//          dc_a = max(0, |wrap(com_a - cg_a)| - hg_a),  l^2 < theta^2 dc^2  and gap^2 > 0
//   leaf   : one particle entry per particle
//   else   : push the children.
//
// A list entry is a node index with kCellTag set (the node's mass at its centre of mass) or
// a particle's position in key order.  The count pass records each group's list length;
// after a prefix sum the emit pass writes the entries.  The traversal order depends only on
// the tree, so both passes visit the same nodes in the same order.
#include "common.hpp"

namespace tpm {
namespace {

constexpr int kStackCap = 1024;

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

struct Visit {
    int kind; // 0 skip, 1 cell entry, 2 leaf particles, 3 open
    uint32_t ne, np, f, cf;
};

// The decision for a node with record w (see the top of this file).
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
    double D = d0 * d0 + d1 * d1 + d2 * d2;
        if (l * l < wp.th2 * D && G > 0.0) {
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

template <int EMIT>
__global__ __launch_bounds__(64) void k_walk(const WalkNode *__restrict__ wn, GroupArrays gr,
                                             uint32_t n_groups,
                                             WalkParams wp, uint64_t *__restrict__ cnt_off,
                                             uint32_t *__restrict__ entries,
                                             unsigned *overflow, uint32_t *__restrict__ gcells)
{
    __shared__ uint32_t stk[kStackCap];
    __shared__ uint32_t s_mark[64];
    const uint32_t g = xcd_block(blockIdx.x, gridDim.x);
    const int lane = threadIdx.x;
    if (g >= n_groups) return;
    const double cg0 = gr.cgx[g], cg1 = gr.cgy[g], cg2 = gr.cgz[g];
    const double hg0 = gr.hgx[g], hg1 = gr.hgy[g], hg2 = gr.hgz[g];
    uint64_t out = EMIT ? cnt_off[g] : 0;
    uint64_t written = 0, ncell = 0;
    if (lane == 0) stk[0] = 0;
    int top = 1;
    __syncthreads();
    while (top > 0) {
        // a popped node pushes at most 8 children: top - k + 8k <= kStackCap
        int room = (kStackCap - top) / 7;
        int k = top < 64 ? top : 64;
        if (room < 1) room = 1;
        if (k > room) k = room;
        Visit a{0, 0u, 0u, 0u, 0u};
        const bool has = lane < k;
        uint32_t u = has ? stk[top - k + lane] : 0u;
        if (u >= wp.n_nodes) { // cannot happen for a well-formed tree: report, never read
            atomicOr(overflow, 2u);
            u = 0u;
        }
        const WalkNode rec = wn[u]; // an idle lane reads the root's record (node 0)
        if (has) a = visit(rec, wp, cg0, cg1, cg2, hg0, hg1, hg2);
        __syncthreads(); // every lane has read its stack slot before the stack is rewritten
        top -= k;
        uint32_t ne_tot, np_tot;
        const uint32_t ne_ex = wave_excl_scan(a.ne, &ne_tot);
        const uint32_t np_ex = wave_excl_scan(a.np, &np_tot);
        if (EMIT && ne_tot) {
            // Expand this step's entries cooperatively so the global writes are contiguous,
            // 64 slots at a time.  Each lane whose run starts inside the chunk marks its
            // start slot with lane + 1; a running maximum over the chunk's slots then names
            // the owner of every slot (the previous chunk's last owner carries over).
            uint32_t carry = 0;
            uint32_t *dst = entries + out + written;
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
                if (q < ne_tot) dst[q] = cell ? v : v + (q - ex);
            }
        }
        written += ne_tot;
        ncell += (uint64_t)__popcll(__ballot(a.kind == 1));
        if (top + (int)np_tot > kStackCap) {
            if (lane == 0) atomicOr(overflow, 1u);
            break;
        }
        if (a.kind == 3)
            for (uint32_t c = 0; c < a.np; ++c) stk[top + np_ex + c] = a.cf + c;
        top += (int)np_tot;
        __syncthreads(); // pushes visible before the next pops
    }
    if (lane == 0) {
        if (!EMIT)
            cnt_off[g] = written;
        else
            gcells[g] = (uint32_t)ncell;
    }
}

// (cell entries, particle entries, interactions = sum_g count_g * L_g): block reductions and
// one atomic per block.
__global__ __launch_bounds__(256) void k_walk_stats(GroupArrays gr, uint32_t n_groups,
                                                    const uint64_t *__restrict__ off,
                                                    const uint32_t *__restrict__ gcells,
                                                    unsigned long long *stats)
{
    unsigned long long c = 0, p = 0, it = 0;
    for (uint32_t g = blockIdx.x * blockDim.x + threadIdx.x; g < n_groups;
         g += gridDim.x * blockDim.x) {
        unsigned long long len = off[g + 1] - off[g];
        c += gcells[g];
        p += len - gcells[g];
        it += len * gr.count[g];
    }
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

void launch_walk(const WalkNode *wn, GroupArrays gr, uint32_t n_groups, WalkParams wp, int emit,
                 uint64_t *counts_or_offsets, uint32_t *entries, unsigned *overflow,
                 uint32_t *gcells, unsigned long long *stats, hipStream_t s)
{
    if (!n_groups) return;
    if (emit) {
        k_walk<1><<<n_groups, 64, 0, s>>>(wn, gr, n_groups, wp, counts_or_offsets, entries,
                                         overflow, gcells);
        unsigned b = (n_groups + 255) / 256;
        k_walk_stats<<<b < 256 ? b : 256, 256, 0, s>>>(gr, n_groups, counts_or_offsets, gcells,
                                                       stats);
    } else {
        k_walk<0><<<n_groups, 64, 0, s>>>(wn, gr, n_groups, wp, counts_or_offsets, entries,
                                         overflow, gcells);
    }
}

} // namespace tpm
