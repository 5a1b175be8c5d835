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

constexpr int kStackCap = 2048;

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
__global__ __launch_bounds__(64) void k_walk(NodeArrays nd, GroupArrays gr, uint32_t n_groups,
                                             WalkParams wp, uint64_t *__restrict__ cnt_off,
                                             uint32_t *__restrict__ entries,
                                             unsigned *overflow, unsigned long long *stats)
{
    __shared__ uint32_t stk[kStackCap];
    const uint32_t g = blockIdx.x;
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
            int lev = nd.level[u];
            double l = wp.lside[lev];
            double half = l * 0.5;
            double v0 = fabs(wrapd(nd.cnx[u] - cg0, L)) - (half + hg0);
            double v1 = fabs(wrapd(nd.cny[u] - cg1, L)) - (half + hg1);
            double v2 = fabs(wrapd(nd.cnz[u] - cg2, L)) - (half + hg2);
            double gp0 = v0 > 0.0 ? v0 : 0.0, gp1 = v1 > 0.0 ? v1 : 0.0,
                   gp2 = v2 > 0.0 ? v2 : 0.0;
            double G = gp0 * gp0 + gp1 * gp1 + gp2 * gp2;
            if (G < rc2) {
                double w0 = fabs(wrapd(nd.comx[u] - cg0, L)) - hg0;
                double w1 = fabs(wrapd(nd.comy[u] - cg1, L)) - hg1;
                double w2 = fabs(wrapd(nd.comz[u] - cg2, L)) - hg2;
                double d0 = w0 > 0.0 ? w0 : 0.0, d1 = w1 > 0.0 ? w1 : 0.0,
                       d2 = w2 > 0.0 ? w2 : 0.0;
                double D = d0 * d0 + d1 * d1 + d2 * d2;
                uint32_t nch = nd.nchild[u];
                if (l * l < th2 * D && G > 0.0) {
                    kind = 1;
                    ne = 1;
                } else if (nch == 0) {
                    kind = 2;
                    f = nd.first[u];
                    ne = nd.count[u];
                } else {
                    kind = 3;
                    cf = nd.child_first[u];
                    np = nch;
                }
            }
        }
        __syncthreads(); // every lane has read its stack slot before the stack is rewritten
        top -= k;
        uint32_t ne_tot, np_tot;
        uint32_t ne_ex = wave_excl_scan(ne, &ne_tot);
        uint32_t np_ex = wave_excl_scan(np, &np_tot);
        if (EMIT) {
            uint64_t at = out + written + ne_ex;
            if (kind == 1) {
                entries[at] = u | kCellTag;
            } else if (kind == 2) {
                for (uint32_t c = 0; c < ne; ++c) entries[at + c] = f + c;
            }
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
        if (!EMIT) {
            cnt_off[g] = written;
        } else {
            atomicAdd(&stats[0], (unsigned long long)ncell);
            atomicAdd(&stats[1], (unsigned long long)(written - ncell));
            atomicAdd(&stats[2], (unsigned long long)(written * gr.count[g]));
        }
    }
}

} // namespace

void launch_walk(NodeArrays nd, GroupArrays gr, uint32_t n_groups, WalkParams wp, int emit,
                 uint64_t *counts_or_offsets, uint32_t *entries, unsigned *overflow,
                 unsigned long long *stats, hipStream_t s)
{
    if (!n_groups) return;
    if (emit)
        k_walk<1><<<n_groups, 64, 0, s>>>(nd, gr, n_groups, wp, counts_or_offsets, entries,
                                         overflow, stats);
    else
        k_walk<0><<<n_groups, 64, 0, s>>>(nd, gr, n_groups, wp, counts_or_offsets, entries,
                                         overflow, stats);
}

} // namespace tpm
