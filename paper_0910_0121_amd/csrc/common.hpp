// Internal declarations shared by the library's translation units (host launchers and the
// small device helpers they need).  Nothing here is part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

namespace tpm {

constexpr int kMaxLevel = 21;             // 21 bits per axis, 63-bit keys
constexpr uint32_t kCellTag = 0x80000000u; // list entry: node index | tag, else sorted index
constexpr int kSortBits = 8;               // radix digit width
constexpr int kSortBins = 1 << kSortBits;
constexpr int kSortThreads = 256;
constexpr int kSortItems = 16;
constexpr int kSortTile = kSortThreads * kSortItems;

// Flags raised by the validation/key kernel.
constexpr unsigned kFlagNonFinite = 1u; // non-finite position or mass, or mass <= 0
constexpr unsigned kFlagRange = 2u;     // position outside [0, L)

// Device arrays of one tree (structure of arrays).  Nodes are stored level by level; the
// children of a node are contiguous and in octant order.
struct NodeArrays {
    uint64_t *code;        // (1 << 3 level) | key prefix
    uint32_t *first;       // first particle (key order)
    uint32_t *count;       // particles
    uint32_t *child_first; // index of the first child
    uint32_t *parent;      // index of the parent (root: itself)
    uint8_t *nchild;       // 0 for a leaf
    uint8_t *level;
    double *mass;          // FP64 moments
    double *comx, *comy, *comz; // mass-weighted position sums (the centre of mass is in nsrc)
    double *cnx, *cny, *cnz; // cube centres ((i + 1/2) * L / 2^level)
    // Sources as 32-byte records, one cache-line sector per list entry:
    double4 *nsrc;        // per node: centre of mass and mass
    const double4 *psrc;  // per particle in key order: position and mass
};

// Everything the walk reads about one node, in one 64-byte record (one cache line), built
// once per tree after the moments.
struct alignas(64) WalkNode {
    double cn[3];  // cube centre
    double com[3]; // centre of mass
    uint32_t first, count, child_first;
    uint8_t level, nchild, pad0, pad1;
};
static_assert(sizeof(WalkNode) == 64, "WalkNode must be one 64-byte line");

struct GroupArrays {
    uint32_t *node, *first, *count;
    double *cgx, *cgy, *cgz;  // bbox centre (lo + hi) / 2
    double *hgx, *hgy, *hgz;  // bbox half size (hi - lo) / 2
    double *xgx, *xgy, *xgz;  // cube centre of the group node (FP32 origin)
    double *lox, *loy, *loz, *hix, *hiy, *hiz;
};

// ------------------------------------------------------------------ launchers (k_scan.hip)
// Exclusive prefix sum in place over n values; the total is written to *total (device).
// tmp must hold scan_tmp_elems(n) values of the same type.
size_t scan_tmp_elems(size_t n);
// Host-visible results without a stream synchronisation: copies up to three runs of device
// words (n0 + n1 + n2 < kMailboxWords in all) into the host-mapped mailbox from word 1 on
// and then writes seq into word 0; the host waits for word 0 to read seq.
constexpr uint32_t kMailboxWords = 64;
void publish_words(const uint32_t *src0, uint32_t n0, const uint32_t *src1, uint32_t n1,
                   const uint32_t *src2, uint32_t n2, uint32_t *mailbox, uint32_t seq,
                   hipStream_t s);
void fill_u32(uint32_t *p, size_t n, uint32_t v, hipStream_t s);
void fill_u64(uint64_t *p, size_t n, uint64_t v, hipStream_t s);
void scan_u32(uint32_t *data, size_t n, uint32_t *total, uint32_t *tmp, hipStream_t s);
void scan_u64(uint64_t *data, size_t n, uint64_t *total, uint64_t *tmp, hipStream_t s);

// ------------------------------------------------------------------ launchers (k_build.hip)
// Also stores each particle's (x, y, z, m) as one 32-byte record for the gather.
void launch_keys(int64_t n, const double *x, const double *y, const double *z, const double *m,
                 double L, uint64_t *key, uint32_t *idx, unsigned *flags, double4 *rec,
                 hipStream_t s);
// Stable LSD radix sort of (key, idx) by key; results end in key/idx.  hist holds
// sort_hist_elems(n) values.
size_t sort_hist_elems(int64_t n);
void radix_sort(int64_t n, uint64_t *key, uint32_t *idx, uint64_t *key_alt, uint32_t *idx_alt,
                uint32_t *hist, uint32_t *scan_tmp, hipStream_t s);
// The sort in two steps: stable passes over bits [kRunBits, 64) only, then each run of equal
// high bits sorted by (key, index) in place.  Returns true if the result is in key_alt /
// idx_alt (an odd number of passes).  long_runs holds long_cap entries; flags (device, two
// words) ends with flags[1] != 0 if a run could not be sorted this way: the order is then
// incomplete and radix_sort (on the returned arrays) must follow.
constexpr int kRunBits = 24;
constexpr uint32_t kShortRun = 8; // the register sorting network in k_fix_runs has 8 inputs
constexpr uint32_t kLongRun = 2048;
bool radix_sort_high(int64_t n, uint64_t *key, uint32_t *idx, uint64_t *key_alt,
                     uint32_t *idx_alt, uint32_t *hist, uint32_t *scan_tmp, uint2 *long_runs,
                     uint32_t long_cap, unsigned *flags, hipStream_t s);
// Writes the key-ordered records psrc (x, y, z, m) and the bit pattern of the largest mass
// into *mmax (the particle mesh scales its fixed-point sums by it).
void launch_permute(int64_t n, const uint32_t *idx, const double4 *rec, double4 *psrc,
                    unsigned long long *mmax, hipStream_t s);
void launch_root(NodeArrays nd, uint32_t n, double L, hipStream_t s);
// Level step: nodes [lo, hi) of level `level`; writes nchild, per-node child counts into
// cnt (hi - lo values) for the scan, and the octant bounds of subdivided nodes into bnd
// (7 (hi - lo) values).  Levels of at most kWideSplitNodes nodes use one wave per node.
constexpr uint32_t kWideSplitNodes = 16384;
void launch_split(NodeArrays nd, const uint64_t *key, uint32_t lo, uint32_t hi, int level,
                  int n_leaf, uint32_t *cnt, uint32_t *bnd, hipStream_t s);
// Emit children of nodes [lo, hi) at base + exclusive prefix in cnt, from the bounds in bnd.
void launch_emit(NodeArrays nd, const uint32_t *bnd, uint32_t lo, uint32_t hi, int level,
                 uint32_t base, const uint32_t *cnt, double L, hipStream_t s);
// Moments of the nodes [lo, hi) of one level, deepest level first: mass, position sums S
// (comx/comy/comz; the centre of mass S / M goes to nsrc and the walk records wn).
// derive = 1 for a tree from launch_tree_emit: nchild and internal counts are set here, the
// children of the level's nodes being the nodes [child_first[lo], child_end).
void launch_moments(NodeArrays nd, const double4 *ps, uint32_t lo, uint32_t hi, int derive,
                    uint32_t child_end, WalkNode *wn, hipStream_t s);
// The octree straight from the sorted keys (n >= 1, n_leaf - 1 <= kTreeWin): the same nodes in
// the same order as the level-by-level split.  launch_tree_levels writes per particle the
// levels of the nodes that start there and its leaf's count (sl, n words), per block of tree_blocks(n) the counts
// per level (blk, kMaxLevel + 1 rows of tree_blocks(n) words, left as exclusive prefixes) and
// the nodes per level into tot (kMaxLevel + 1 words).  With off[] from tot, launch_tree_emit
// writes every node but nchild and the internal counts (left to the moments with derive = 1).
constexpr int kTreeWin = 256;
struct TreeOffsets {
    uint32_t off[kMaxLevel + 3]; // first node of each level; off[22] = off[23] = node count
};
uint32_t tree_blocks(int64_t n);
void launch_tree_levels(const uint64_t *key, uint32_t n, int n_leaf, uint32_t *sl, uint32_t *blk,
                        uint32_t *tot, hipStream_t s);
void launch_tree_emit(NodeArrays nd, const uint64_t *key, const uint32_t *sl, const uint32_t *blk,
                      const TreeOffsets &to, uint32_t n, double L, hipStream_t s);
// Groups: mark in gstart[first] (n values, zeroed here) every maximal node with
// count <= n_crit or no children; then compact in key order.
void launch_group_mark(NodeArrays nd, uint32_t n_nodes, int n_crit, uint32_t *gstart,
                       uint32_t *gflag, int64_t n, hipStream_t s);
void launch_group_compact(const uint32_t *gstart, const uint32_t *gpos, int64_t n,
                          uint32_t *gnode, hipStream_t s);
// Also lowers *min_level to the shallowest group level and raises *max_count to the
// largest group.
void launch_group_bbox(NodeArrays nd, GroupArrays gr, uint32_t n_groups, const double4 *ps,
                       unsigned *min_level,
                       unsigned *max_count, hipStream_t s);

// ------------------------------------------------------------------ launchers (k_walk.hip)
// open = 0: fixed angle, th2 = theta^2.  open = 1: theta(d) of eq. (12) from eta = r_cut/2,
// theta0 and the cap theta_max; th2 = theta_max^2 and th2lo = theta_lo^2, where theta_lo =
// min(theta_max, theta0 / sqrt(0.46)) is below every value theta(d) takes (R g(R) peaks at
// 0.45273 near R = 0.650).
struct WalkParams {
    double L, rc2, th2, th2lo;
    double eta, theta0, theta_max;
    uint32_t n_nodes;
    uint32_t open;
};
// Group g's interaction list is entries[off[g] .. off[g] + len[g]).
// Two passes: the count pass writes each list length to counts[g]; after the caller's prefix
// sum (counts -> off) the emit pass writes the lists, len and gcells (cell entries).
void launch_walk_count(const WalkNode *wn, GroupArrays gr, uint32_t n_groups, WalkParams wp,
                       uint64_t *counts, unsigned *overflow, hipStream_t s);
void launch_walk_emit(const WalkNode *wn, GroupArrays gr, uint32_t n_groups, WalkParams wp,
                      const uint64_t *off, uint32_t *len, uint32_t *entries, unsigned *overflow,
                      uint32_t *gcells, hipStream_t s);
// One pass: n_waves waves write the lists into chunks of `chunk` entries taken from the
// pool entries[0, pool_cap); a group is walked into the wave's current chunk if at least
// `reserve` entries are left there, else (or if it did not fit) into a fresh chunk.  Sets bit 4 of *overflow if a list or the pool ran out of room
// (the lists are then incomplete).  counters holds kXcds + 2 words (8-byte aligned).
void launch_walk_pool(const WalkNode *wn, GroupArrays gr, uint32_t n_groups, WalkParams wp,
                      uint32_t n_waves, uint64_t pool_cap, uint64_t chunk, uint64_t reserve,
                      uint32_t *counters, uint64_t *off, uint32_t *len, uint32_t *entries,
                      unsigned *overflow, uint32_t *gcells, hipStream_t s);
// Adds (cell entries, particle entries, interactions) into stats[0..2] and the longest list
// into stats[3] (all zeroed by the caller).
void launch_walk_stats(GroupArrays gr, uint32_t n_groups, const uint32_t *len,
                       const uint32_t *gcells, unsigned long long *stats, hipStream_t s);

// Shared launches over several boxes.  The groups of boxes 0 .. nb-1 are laid end to end as
// one sequence of work items; box b holds items [g0, g0 + n_groups).  Each box keeps its own
// tree, lists and flags, exactly as in a walk of that box alone.
constexpr int kMaxBatch = 16;
struct WalkBox {
    const WalkNode *wn;
    GroupArrays gr;
    WalkParams wp;
    uint64_t *off;                 // counts (count pass) or list offsets
    uint32_t *len, *entries, *gcells;
    unsigned long long *pool_next; // one-pass walk: the box's pool counter
    uint64_t pool_cap, chunk, reserve;
    unsigned *overflow;
    uint32_t g0, n_groups;
};
// The two passes over all items of the boxes (one wave per item; descriptors in device
// memory, total = sum of n_groups).
void launch_walk_count_multi(const WalkBox *boxes, int nb, uint32_t total, hipStream_t s);
void launch_walk_emit_multi(const WalkBox *boxes, int nb, uint32_t total, hipStream_t s);
// One pass over all items: n_waves waves take items in batches from kXcds counters (zeroed
// here; counters holds kXcds words) and write each box's lists into chunks of that box's
// pool.  A box whose list or pool runs out of room gets bit 4 of its overflow flag; the other
// boxes are not affected.
void launch_walk_pool_multi(const WalkBox *boxes, int nb, uint32_t total, uint32_t n_waves,
                            uint32_t *counters, hipStream_t s);

// ------------------------------------------------------------------ launchers (k_force.hip)
// Workgroups are dealt to the 8 XCDs (each with its own L2) round-robin by block index.
// xcd_block renumbers block b of n so that each XCD takes a contiguous run: neighbouring
// groups (key order) then share one L2.  A bijection on [0, n).
constexpr uint32_t kXcds = 8;
__device__ __forceinline__ uint32_t xcd_block(uint32_t b, uint32_t n)
{
    const uint32_t q = n / kXcds, r = n % kXcds, x = b % kXcds;
    return x * q + (x < r ? x : r) + b / kXcds;
}

struct ForceParams {
    double L, eps2, inv_eta, eta, rc2, rc;
    uint32_t *kept; // per group, list entries that survived the cutoff cull
};

// The FP32 pair law G(s) = g(2 sqrt(s)) / (s + (eps/r_cut)^2)^(3/2) (s = r^2 in units of
// r_cut^2) as cubic pieces in u = min(s + c, 1): 2^kTabSegBits pieces per octave of u,
// located by the bit pattern of u (index = (bits >> kTabShift) - base, position = the low
// kTabShift bits), from u = c up to u = 1 (R = 2); the last entry is zero and takes u = 1.
constexpr int kTabSegBits = 5;
constexpr int kTabShift = 23 - kTabSegBits;
constexpr uint32_t kTabMaxEntries = 1025; // 32 octaves: eps / r_cut down to 2^-13
struct ForceTable {
    const float4 *coef; // entries x (c0, c1, c2, c3), device
    uint32_t entries;
    uint32_t base;      // (bit pattern of c) >> kTabShift
    float c;            // a power of two at most (eps/r_cut)^2 / 64
};
// Fills the table for eps / r_cut (host, FP64 fit, rounded to float); false if eps / r_cut is
// not positive or too small for kTabMaxEntries entries.
bool build_force_table(double eps_over_rcut, std::vector<float4> &coef, uint32_t &base, float &c);

constexpr int kForceClasses = 8; // FP32 force: one class per blocking factor K = 1..8
// Layout of the class buffer (u32 words): the class sizes, per class the kXcds + 1 part
// starts (absolute word positions in the buffer), the per-(class, part) queue counters, the
// (class, part, cost bucket) cursors, then per class its group ids (stride words apart),
// each part longest first.
constexpr uint32_t kClsCounts = 0;
constexpr uint32_t kClsStarts = kClsCounts + kForceClasses;
constexpr uint32_t kClsQueue = kClsStarts + kForceClasses * (kXcds + 1);
constexpr uint32_t kClsBins = kClsQueue + kForceClasses * kXcds;
constexpr uint32_t kClsLists = kClsBins + kForceClasses * kXcds * 64;
// Classes, parts and longest-first order of the groups (len: list lengths), into cls.
void launch_classify(GroupArrays gr, uint32_t n_groups, const uint32_t *len, uint32_t *cls,
                     uint32_t stride, hipStream_t s);
// Empties the force queues (a fill kernel): on the call's stream before the class launches
// fork onto the other streams.
void launch_force_f32_prep(uint32_t *cls, hipStream_t s);
// class_counts: host copy of the class sizes.  Classes are launched largest blocking factor
// first, round-robin over the n_streams streams (the caller forks and joins them); each is a
// persistent kernel of at most n_cu x (its waves per SIMD) workgroups.
void launch_force_f32(NodeArrays nd, GroupArrays gr, uint32_t *cls, const uint32_t *class_counts,
                      const uint64_t *off, const uint32_t *len, const uint32_t *entries,
                      const double4 *ps, const uint32_t *pidx, ForceParams fp, ForceTable ft,
                      void *rec, int rec64, int n_cu, const hipStream_t *streams,
                      int n_streams);
// The FP32 force of several boxes in one persistent launch per class: box b's class buffer,
// lists and records as launch_force_f32 takes them for that box alone (queues zeroed by
// launch_force_f32_prep).  Boxes whose tables have equal tab_id share one LDS copy; a
// workgroup reloads the table when the next box's differs.  class_totals[K - 1] is the sum
// over boxes of class K's size, max_entries the largest table.  float4 records only.
struct ForceBox {
    NodeArrays nd;
    GroupArrays gr;
    uint32_t *cls;
    const uint64_t *off;
    const uint32_t *len, *entries;
    const double4 *ps;
    const uint32_t *pidx;
    ForceParams fp;
    ForceTable ft;
    void *rec;
    uint64_t tab_id;
};
void launch_force_f32_multi(const ForceBox *boxes, int nb, const uint32_t *class_totals,
                            uint32_t max_entries, int n_cu, const hipStream_t *streams,
                            int n_streams);
// rec of the force launchers: one record per particle in the caller's order (pidx), float4
// (ax, ay, az, 0) or, with rec64, double4.  launch_force_out then writes them out: mode 0
// float arrays, 1 double arrays (from float4 / double4 records), 2 kick (v += dt a into double
// velocities, double4 records), walking the records in order.
void launch_force_out(const void *rec, int mode, int64_t n, void *ax, void *ay, void *az,
                      double dt, hipStream_t s);
// FP32 pair routine on explicit positions, pair by pair (xg: host, 3 values).
void launch_pairwise_f32(int64_t n_i, const double *xi, int64_t n_j, const double *xj,
                         const double *mj, const double *xg, double eta, ForceTable ft,
                         double *out, hipStream_t s);
// sum over groups of count * kept (pairs the force kernel evaluated) into *out (device).
void launch_kept_stats(GroupArrays gr, uint32_t n_groups, const uint32_t *kept,
                       unsigned long long *out, hipStream_t s);
void launch_force_f64(NodeArrays nd, GroupArrays gr, uint32_t n_groups, const uint64_t *off,
                      const uint32_t *len, const uint32_t *entries, const double4 *ps, const uint32_t *pidx,
                      ForceParams fp, void *rec, int rec64, hipStream_t s);

// Particle-mesh long-range force (k_pm.hip), mesh N^3 with N a power of two in [16, 1024].
// Lines per FFT workgroup for mesh size N.
int pm_bundle_lines(int N);
// Octant table of the Green's function ((N/2+1)^3 floats) and N/2 twiddles.
void launch_pm_green(int N, double L, double eta, float *green, float2 *tw, hipStream_t s);
// Fills the fixed-point mass mesh (N^3 words, every word written) from the key-ordered records
// and their sorted keys; mx holds the largest mass.  Scratch: cell_start (cells + 1 words),
// item_start (cells + 1 words), scan_tmp (scan_tmp_elems(cells) words) and slots
// (pm_assign_items_max x pm_assign_slot_words() words), cells = pm_assign_cells(N).
size_t pm_assign_cells(int N);
size_t pm_assign_items_max(int N, int64_t n);
size_t pm_assign_slot_words();
void launch_pm_assign(const double4 *ps, const uint64_t *key, int64_t n, int N, double L,
                      const unsigned long long *mx, uint32_t *cell_start, uint32_t *item_start,
                      uint32_t *scan_tmp, unsigned long long *slots, unsigned long long *mass,
                      hipStream_t s);
// Potential phi (N^3 floats) from the mass mesh, through the complex work mesh grid.
void launch_pm_potential(const unsigned long long *mass, const unsigned long long *mx,
                         int64_t n, int N, float2 *grid, float *phi, const float *green,
                         const float2 *tw, hipStream_t s);
// Mesh force (N^3 float4: Fx, Fy, Fz, 0) from phi.
void launch_pm_force(const float *phi, int N, double L, float4 *f, hipStream_t s);
// Interpolated force of key-ordered particle k (ps[k]) into stage[idx[k]] = (ax, ay, az, 0),
// i.e. in the caller's order (idx is the sort permutation).  cell_start and item_start as
// launch_pm_assign left them for the same particles.
void launch_pm_interp(const double4 *ps, int64_t n, int N, double L, const float4 *f,
                      const uint32_t *idx, float4 *stage, const uint32_t *cell_start,
                      const uint32_t *item_start, hipStream_t s);
// ax[o] = stage[o].x etc. (float or double; accumulate adds).
void launch_pm_split(const float4 *stage, int64_t n, void *ax, void *ay, void *az,
                     int out_fp64, int accumulate, hipStream_t s);

// Quadrupole terms of the cell entries (k_quad.hip).  Q: 6 doubles per node (xx, yy, zz,
// xy, xz, yz about the centre of mass), filled level by level from the deepest.
void launch_second_moments(NodeArrays nd, const double4 *ps, uint32_t lo, uint32_t hi,
                           double *Q, hipStream_t s);
// Adds the cells' second-order terms to the force records (caller's order, float4 or, with
// rec64, double4), computed in FP64 (fp64_math) or FP32.
void launch_quad(NodeArrays nd, GroupArrays gr, uint32_t n_groups, const uint64_t *off,
                 const uint32_t *len, const uint32_t *entries, const double4 *ps,
                 const uint32_t *pidx, const double *Q, ForceParams fp, void *rec,
                 int fp64_math, int rec64, hipStream_t s);

// Time stepping (k_step.hip).  Accelerations are float (acc_fp64 = 0) or double arrays.
// out receives the bit pattern of min_i(sqrt(eps / |a_i|), eps / |v_i|) (+inf if none binds).
void launch_timestep(int64_t n, const double *vx, const double *vy, const double *vz,
                     const void *ax, const void *ay, const void *az, int acc_fp64, double eps,
                     unsigned long long *out, hipStream_t s);
// Device scratch of the allocation-free time step (a static device array, 256 bytes): its
// address on `device`, which must be the current device, looked up once per device.
constexpr int kStepScratchWords = 32;
constexpr int kMaxDevices = 64;
hipError_t step_scratch(int device, unsigned long long **out);
// v += a dt_kick, then x += v dt_drift wrapped into [0, L), in place.
void launch_kick_drift(int64_t n, double *x, double *y, double *z, double *vx, double *vy,
                       double *vz, const void *ax, const void *ay, const void *az, int acc_fp64,
                       double dt_kick, double dt_drift, double L, hipStream_t s);

} // namespace tpm
