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

__device__ __forceinline__ double wrapd(double v, double L)
{
    double h = 0.5 * L;
    if (v >= h) return v - L;
    if (v < -h) return v + L;
    return v;
}

__device__ __forceinline__ uint32_t wave_excl_scan(uint32_t v, uint32_t *total)
{
    const int lane = threadIdx.x & 63;
    uint32_t inc = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        uint32_t o = __shfl_up(inc, d, 64);
        if (lane >= d) inc += o;
    }
    *total = __shfl(inc, 63, 64);
    return inc - v;
}

template <int EMIT>
__global__ __launch_bounds__(64) void k_walk(const WalkNode *__restrict__ wn, GroupArrays gr,
                                             uint32_t n_groups,
                                             WalkParams wp, uint64_t *__restrict__ cnt_off,
                                             uint32_t *__restrict__ entries,
                                             unsigned *overflow, uint32_t *__restrict__ gcells)
{
    __shared__ uint32_t stk[kStackCap];
    __shared__ uint32_t s_ex[64], s_val[64];
    __shared__ uint8_t s_cell[64];
    const uint32_t g = xcd_block(blockIdx.x, gridDim.x);
    const int lane = threadIdx.x;
    if (g >= n_groups) return;
    const double L = wp.L, rc2 = wp.rc2, th2 = wp.th2;
    const double cg0 = gr.cgx[g], cg1 = gr.cgy[g], cg2 = gr.cgz[g];
    const double hg0 = gr.hgx[g], hg1 = gr.hgy[g], hg2 = gr.hgz[g];
    uint64_t out = EMIT ? cnt_off[g] : 0;
    uint64_t written = 0, ncell = 0;
    if (lane == 0) stk[0] = 0;
    int top = 1;
    __syncthreads();
    while (top > 0) {
        int room = (kStackCap - top) / 8;
        int k = top < 64 ? top : 64;
        if (room < 1) room = 1;
        if (k > room) k = room;
        uint32_t u = 0;
        int kind = 0; // 0 skip, 1 cell entry, 2 leaf particles, 3 open
        uint32_t ne = 0, np = 0, f = 0, cf = 0;
        if (lane < k) {
            u = stk[top - k + lane];
            const WalkNode w = wn[u];
            int lev = w.level;
            double l = wp.lside[lev];
            double half = l * 0.5;
            double v0 = fabs(wrapd(w.cn[0] - cg0, L)) - (half + hg0);
            double v1 = fabs(wrapd(w.cn[1] - cg1, L)) - (half + hg1);
            double v2 = fabs(wrapd(w.cn[2] - cg2, L)) - (half + hg2);
            double gp0 = v0 > 0.0 ? v0 : 0.0, gp1 = v1 > 0.0 ? v1 : 0.0,
                   gp2 = v2 > 0.0 ? v2 : 0.0;
            double G = gp0 * gp0 + gp1 * gp1 + gp2 * gp2;
            if (G < rc2) {
                double w0 = fabs(wrapd(w.com[0] - cg0, L)) - hg0;
                double w1 = fabs(wrapd(w.com[1] - cg1, L)) - hg1;
                double w2 = fabs(wrapd(w.com[2] - cg2, L)) - hg2;
                double d0 = w0 > 0.0 ? w0 : 0.0, d1 = w1 > 0.0 ? w1 : 0.0,
                       d2 = w2 > 0.0 ? w2 : 0.0;
                double D = d0 * d0 + d1 * d1 + d2 * d2;
                uint32_t nch = w.nchild;
                if (l * l < th2 * D && G > 0.0) {
                    kind = 1;
                    ne = 1;
                } else if (nch == 0) {
                    kind = 2;
                    f = w.first;
                    ne = w.count;
                } else {
                    kind = 3;
                    cf = w.child_first;
                    np = nch;
                }
            }
        }
        __syncthreads(); // every lane has read its stack slot before the stack is rewritten
        top -= k;
        uint32_t ne_tot, np_tot;
        uint32_t ne_ex = wave_excl_scan(ne, &ne_tot);
        uint32_t np_ex = wave_excl_scan(np, &np_tot);
        if (EMIT && ne_tot) {
            // Expand this step's entries cooperatively so the global writes are contiguous:
            // slot q belongs to the last lane whose exclusive offset is <= q.
            s_ex[lane] = ne_ex;
            s_val[lane] = kind == 1 ? (u | kCellTag) : f;
            s_cell[lane] = kind == 1;
            __syncthreads();
            uint32_t *dst = entries + out + written;
            for (uint32_t q = lane; q < ne_tot; q += 64) {
                int lo = 0, hi = 63;
                while (lo < hi) {
                    int mid = (lo + hi + 1) >> 1;
                    if (s_ex[mid] <= q)
                        lo = mid;
                    else
                        hi = mid - 1;
                }
                uint32_t v = s_val[lo];
                dst[q] = s_cell[lo] ? v : v + (q - s_ex[lo]);
            }
            __syncthreads();
        }
        written += ne_tot;
        ncell += (uint64_t)__popcll(__ballot(kind == 1));
        if (top + (int)np_tot > kStackCap) {
            if (lane == 0) atomicOr(overflow, 1u);
            break;
        }
        if (kind == 3)
            for (uint32_t c = 0; c < np; ++c) stk[top + np_ex + c] = cf + c;
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
