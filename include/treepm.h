/*
 * treepm.h -- C ABI of the MI355X short-range TreePM tree force.
 *
 * The library computes the particle-particle (short-range) part of the TreePM force of
 * Ishiyama, Fukushige & Makino, "GreeM: Massively Parallel TreePM Code for Large
 * Cosmological N-body Simulations" (PASJ 2009, arXiv:0910.0121), for one periodic box held
 * on one GPU:
 *
 *   a_i = sum over the interaction list of i's group of
 *         m_j d g_P3M(|d|/eta) / (|d|^2 + eps^2)^(3/2),   d = x_j - x_i (nearest image),
 *
 * with the cutoff function g_P3M of eq. (2), 2 eta = r_cut (Section 2.1, eq. 1; Section 2.2
 * step 1 sets r_cut = 3 / N_PM), Plummer softening eps (Section 2.4), and the lists built by
 * Barnes' group walk over a Morton-key octree (Section 2.2 steps 2 and 5; Section 3.1.2 for
 * N_leaf and N_crit).  Sources are particles or tree nodes (mass and centre of mass).
 * Accelerations point toward the sources; G = 1.
 *
 * Conventions for every call:
 *  - Return value: TREEPM_OK (0), TREEPM_PENDING (1, ensemble poll only) or a negative
 *    TREEPM_ERR_* code.  No C++ exception or abort crosses this interface.  The text of the
 *    last error of a context is returned by treepm_last_error().
 *  - Memory kinds: TREEPM_HOST buffers are ordinary host memory; TREEPM_DEVICE buffers are
 *    device pointers on the context's GPU.  All buffers are owned by the caller.  Inputs are
 *    copied or read by the library before the call's work completes on the stream.
 *  - Streams: hip_stream is a hipStream_t (NULL = the default stream).  Calls on one context
 *    are stream-ordered and must be made from one thread at a time.  Calls that return
 *    results to host memory synchronise the stream before returning.
 *  - Handles are owned by the library until the matching *_destroy call.
 */
#ifndef TREEPM_H
#define TREEPM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    TREEPM_OK = 0,
    TREEPM_PENDING = 1,
    TREEPM_ERR_ARG = -1,        /* invalid parameter or argument                          */
    TREEPM_ERR_RANGE = -2,      /* a position outside [0, L): the caller must wrap          */
    TREEPM_ERR_OOM = -3,        /* device memory (or the ensemble's HBM budget) exhausted   */
    TREEPM_ERR_DEVICE = -4,     /* a HIP runtime error                                      */
    TREEPM_ERR_STATE = -5,      /* call out of order (walk before build, force before walk) */
    TREEPM_ERR_QUEUE_FULL = -6, /* ensemble request queue full                              */
    TREEPM_ERR_OVERFLOW = -7    /* an internal capacity was exceeded (see last_error)       */
};

enum { TREEPM_FP32 = 0, TREEPM_FP64 = 1 };   /* pair-kernel / output precision */
enum { TREEPM_HOST = 0, TREEPM_DEVICE = 1 }; /* memory kind of caller buffers  */
enum { TREEPM_OPEN_FIXED = 0, TREEPM_OPEN_DISTANCE = 1 }; /* opening criterion        */

/* Parameters of one box (Section 2.2 step 1; Section 2.4; Section 3.1.2).
 *   L        periodic box side, > 0 (the paper normalises it to 1).
 *   mesh     PM mesh spacing L / N_PM, > 0.
 *   r_cut    cutoff radius, 0 < r_cut <= L/2, and r_cut = 3 mesh to relative 1e-12
 *            (2 eta = r_cut = 3 / N_PM).
 *   eps      Plummer softening, >= 0; the FP32 kernel requires eps >= 2^-13 r_cut
 *            (its pair law is tabulated per box for eps / r_cut).
 *   theta    opening angle, 0 <= theta <= 1.  A node of side l is used as one source when
 *            l < theta d, d = distance from its centre of mass to the group's bounding box
 *            (minimum image), and its cube does not touch that box.  Under
 *            TREEPM_OPEN_DISTANCE this is theta_0 of the distance-dependent angle.
 *   n_leaf   a node is subdivided iff it holds >= n_leaf particles (and level < 21); >= 2.
 *   n_crit   groups are the maximal nodes holding <= n_crit particles (or leaves); >= 1;
 *            0 selects the library default (128).
 *   precision TREEPM_FP32: pair force in FP32 on positions relative to the group's cube
 *            centre with compensated accumulation (Section 3.1.1); TREEPM_FP64: plain FP64.
 *            The tree, moments and every walk decision are FP64 in both cases.
 *   opening  TREEPM_OPEN_FIXED (0, the default of a zeroed struct): theta as above.
 *            TREEPM_OPEN_DISTANCE: the distance-dependent angle of Section 4.1, eq. (12),
 *            theta(d) = min(theta_max, theta / sqrt(R g_P3M(R))), R = d / eta (distance in
 *            units of eta), and theta(d) = theta_max where R g(R) = 0 (d = 0 or d >= r_cut);
 *            the node is used when l < theta(d) d.  sqrt and divisions are correctly rounded,
 *            so the lists equal a plain FP64 evaluation.
 *   theta_max the cap of theta(d), 0 <= theta_max <= 1 (read only under
 *            TREEPM_OPEN_DISTANCE).
 *   quadrupole 0 (default): a cell entry is its mass at its centre of mass.  1: it also adds
 *            its second-order term (Section 4.1), (Q d) u + (1/2) tr(Q) d u + (1/2)(d.Q.d) d w
 *            with Q the node's second moment about its centre of mass (FP64, from the
 *            build), d the displacement to the centre of mass, u = h'/r, w = (h'/r)'/r and
 *            h(r) = g_P3M(r/eta) (r^2+eps^2)^(-3/2): the derivatives of the cutoff function
 *            enter through h.  Computed in the force call's precision; the lists are the
 *            same.  Costs 48 bytes per node and a second pass over the cell entries. */
typedef struct {
    double L;
    double mesh;
    double r_cut;
    double eps;
    double theta;
    int32_t n_leaf;
    int32_t n_crit;
    int32_t precision;
    int32_t opening;
    double theta_max;
    int32_t quadrupole;
} treepm_params;

typedef struct treepm_ctx treepm_ctx; /* one resident box on one GPU */
typedef struct treepm_ens treepm_ens; /* ensemble server            */

/* Counts and timings of the last build/walk/force of a context. */
typedef struct {
    int64_t n;              /* particles                                                  */
    int64_t n_nodes;        /* tree nodes                                                 */
    int64_t n_groups;       /* groups (one interaction list each)                         */
    int64_t n_cell_entries; /* list entries that are tree nodes                           */
    int64_t n_part_entries; /* list entries that are particles                            */
    int64_t interactions;   /* sum over groups of (group size x list length)              */
    int32_t max_level;      /* deepest tree level                                         */
    int32_t max_group;      /* largest group                                              */
    double t_ms[4];         /* device time of build, walk, force, and their sum (ms);
                               0 unless timing is enabled with treepm_set_timing          */
    int64_t evaluated;      /* pairs the last force call evaluated: both force kernels
                               skip list entries whose source lies at least r_cut from
                               the group's bounding box (every pair they form adds
                               exactly zero), so this is at most interactions            */
    double latency_ms;      /* ensemble results only: completion minus submission (ms)    */
    double queue_ms;        /* ensemble results only: start of service minus submission,
                               the part of latency_ms spent queued (ms)                  */
    double stage_ms[3];     /* ensemble results only, the service time in three parts
                               (ms): context, input copy and build; wait for a batch;
                               the batch's walk, force and copy of the results to host  */
    int32_t batch_boxes;    /* ensemble results only: boxes whose walk and force shared
                               launches with this request's (1 when it ran alone)        */
    int32_t reserved_;
} treepm_stats;

/* Create a context for one box on HIP device `device`.  Validates *params (ERR_ARG).  The
 * context allocates device memory lazily and keeps it for later calls. */
int treepm_create(const treepm_params *params, int device, treepm_ctx **out);

/* Release every resource of the context, after waiting for its queued work.  NULL is
 * accepted.  Its device buffers, streams and events are kept by the library (per device,
 * process-wide) for later contexts rather than handed back to the driver: a server that
 * evicts and creates boxes continuously then neither frees nor maps device memory while
 * other boxes run.  At most a quarter of the device's memory is kept that way (the rest is
 * freed); treepm_release_cached gives it back. */
int treepm_destroy(treepm_ctx *ctx);

/* Give the device memory that destroyed contexts left for reuse on `device` back to the
 * driver, waiting for any queued work that may still use it.  Contexts alive on the device
 * keep their own buffers.  Returns TREEPM_ERR_DEVICE for a device that does not exist. */
int treepm_release_cached(int device);

/* Replace the parameters of an existing context (same validation as create).  The next
 * call must be treepm_build. */
int treepm_set_params(treepm_ctx *ctx, const treepm_params *params);

/* Record per-phase device times into treepm_stats.t_ms (adds event records to the stream). */
int treepm_set_timing(treepm_ctx *ctx, int enable);

/* How treepm_walk (and treepm_force_short_batch) write a context's lists.  TREEPM_WALK_AUTO
 * (the default): in one pass once an earlier walk has sized the device memory, if the box has
 * at least 98,304 groups (16 per wave of the one-pass launch: below that the launch cannot
 * fill the device and the two passes, a wave per group each, are faster); in two passes
 * otherwise.  TREEPM_WALK_ONE_PASS: in one pass whenever an earlier walk sized it.
 * TREEPM_WALK_TWO_PASS: always in two passes.  The lists are the same in every mode.
 * ERR_ARG for another mode. */
enum { TREEPM_WALK_AUTO = 0, TREEPM_WALK_ONE_PASS = 1, TREEPM_WALK_TWO_PASS = 2 };
int treepm_set_walk_passes(treepm_ctx *ctx, int mode);

/* Build the tree of n particles (Section 2.2 step 2): validate, compute 63-bit Morton keys,
 * stable radix sort, gather positions and masses into key order, build the octree with the
 * N_leaf rule, FP64 node masses and centres of mass, and the N_crit groups.
 * x, y, z, m: n doubles each, of kind mem_kind.  Requires 0 <= x < L on each axis
 * (ERR_RANGE otherwise), finite values and m > 0 (ERR_ARG).  A failed build leaves the
 * context empty. */
int treepm_build(treepm_ctx *ctx, int64_t n, const double *x, const double *y, const double *z,
                 const double *m, int mem_kind, void *hip_stream);

/* Barnes' group walk (Section 2.2 step 5): one interaction list per group.  Requires a
 * build (ERR_STATE).  Fills *stats if non-NULL.  The first walk on a context counts the lists
 * and then writes them (two passes); later walks of boxes with at least 98,304 groups (see
 * treepm_set_walk_passes) write them in one pass into device memory sized from the previous
 * walk (about 1.25x its lists plus a chunk per wave) and fall back to two passes if that is
 * too small, so the lists never depend on the estimate.  ERR_OVERFLOW if a group's traversal
 * stack would exceed its capacity (see last_error). */
int treepm_walk(treepm_ctx *ctx, void *hip_stream, treepm_stats *stats);

/* Short-range force on every particle from its group's list (eq. 1, 2), written in the
 * caller's original particle order.  TREEPM_FP32 boxes work in lengths of r_cut, relative to
 * the group's cube centre: with s = (r / r_cut)^2 the pair law
 * G(s) = g_P3M(2 sqrt(s)) / (s + (eps/r_cut)^2)^(3/2) is G = (1 - s)^4 H(u), u = min(s + c, 1),
 * c a power of two at most (eps/r_cut)^2 / 64, and H comes from a table of cubic pieces built
 * on the host for the box (32 per octave of u, relative least-squares fits, zero at u = 1);
 * the rest of the pair arithmetic is FP32.  ax, ay, az: n values each of type out_prec
 * (TREEPM_FP32 = float, TREEPM_FP64 = double) and kind mem_kind.  Requires a walk
 * (ERR_STATE).  Uses no memory beyond what the build and walk allocated (device outputs). */
int treepm_force_short(treepm_ctx *ctx, void *ax, void *ay, void *az, int out_prec,
                       int mem_kind, void *hip_stream);

/* Walk (as treepm_walk) and FP32 short-range force (as treepm_force_short with float outputs)
 * of n_boxes built boxes at once, with shared launches (Section 2.2 steps 5 and 6 for every
 * box): one traversal launch over the (box, group) pairs of all boxes, and one persistent
 * force launch per size class over all of them.  Each box keeps its own particles, tree,
 * lists and pair-law table, and its results equal, bit for bit, those of treepm_walk followed
 * by treepm_force_short on that box alone.  ctxs: n_boxes (1 .. 16) distinct contexts on one
 * device, each built (ERR_STATE) with precision TREEPM_FP32 (ERR_ARG); ax[b], ay[b], az[b]:
 * box b's n floats each, of kind mem_kind.  The first box's streams and scratch serve the
 * launches.  Returns when host outputs are written (TREEPM_HOST) or the work is queued
 * (TREEPM_DEVICE).  On an error every box is left built but not walked; the failing box's
 * last_error names the cause and the others' say that another box failed. */
int treepm_force_short_batch(treepm_ctx *const *ctxs, int n_boxes, float *const *ax,
                             float *const *ay, float *const *az, int mem_kind,
                             void *hip_stream);

/* The short-range kick fused with the force (Section 2.2 step 5: a particle's velocity is
 * kicked with its short-range force as soon as that is computed, without storing it):
 * v_i += dt a_i for every particle, a_i the acceleration treepm_force_short would give.
 * vx, vy, vz: n doubles each, device arrays on the context's GPU in the caller's particle
 * order (ERR_ARG for host memory); each product dt a_i and each sum is rounded on its own, so
 * the result equals v + dt a with a from treepm_force_short(..., TREEPM_FP64, ...) bit for bit.
 * Requires a walk (ERR_STATE); not for quadrupole boxes (ERR_ARG).  Stream-ordered. */
int treepm_kick_short(treepm_ctx *ctx, double *vx, double *vy, double *vz, double dt,
                      void *hip_stream);

/* Long-range (particle-mesh) acceleration of every particle of the built box (Section 2.2
 * step 1; the long-range half of the split of Section 2.1), on the mesh N_PM = L / mesh,
 * which must be a power of two in [16, 1024] (ERR_ARG otherwise):
 *   - TSC assignment of the masses onto the N_PM^3 mesh points x = i h, h = L / N_PM (the
 *     nearest point and its two neighbours per axis, periodic), summed in 64-bit fixed point;
 *   - potential phi = (1/L^3) sum_{k != 0} G(k) M^(k) e^{ikx} by FFT, with
 *     G(k) = -4 pi S2^(k eta)^2 / (k^2 W(k)^2): the force between two S2 clouds of radius eta
 *     (the complement of eq. 2's cutoff, eta = r_cut / 2) over the TSC window
 *     W = prod_a sinc^3(k_a h / 2), divided out for assignment and interpolation;
 *   - mesh force by fourth-order central differences of -grad phi, then TSC interpolation.
 * Mesh arithmetic is FP32.  Results go to ax/ay/az in the caller's particle order, as
 * out_prec (TREEPM_FP32 = float, TREEPM_FP64 = double) of kind mem_kind; accumulate = 1 adds
 * to the values the arrays hold (so short-range + long-range needs no extra array), 0
 * overwrites them.  Requires a build (ERR_STATE).  Device memory: about 32 N_PM^3 bytes,
 * kept by the context. */
int treepm_force_long(treepm_ctx *ctx, void *ax, void *ay, void *az, int out_prec,
                      int mem_kind, int accumulate, void *hip_stream);

/* ------------------------------------------------------------ time stepping
 * Section 2.2 kicks the velocities with the forces and drifts the positions; Section 2.4 gives
 * the shared adaptive step (eq. 7) and the softening schedule (eq. 6).  Positions, velocities
 * (double) and accelerations (float or double, acc_prec) are device arrays of n particles in
 * the caller's order; these calls use the context's device and L and do not need a build.
 * Arithmetic is FP64 without contraction (plain IEEE evaluation of each formula). */

/* Physical Plummer softening at redshift z, eq. (6): eps_fin (1 + z_crit) / (1 + z) for
 * z >= z_crit, else eps_fin (so the comoving softening is constant before z_crit). */
double treepm_eps_of_z(double z, double eps_fin, double z_crit);

/* Shared time step, eq. (7): *dt = zeta min_i(sqrt(eps / |a_i|), eps / |v_i|), where a term
 * with a zero denominator does not bind (+inf if none does).  eps, zeta finite and > 0.
 * Synchronises the stream. */
int treepm_timestep(treepm_ctx *ctx, int64_t n, const double *vx, const double *vy,
                    const double *vz, const void *ax, const void *ay, const void *az,
                    int acc_prec, double eps, double zeta, void *hip_stream, double *dt);

/* treepm_timestep for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): same arguments, checks and
 * result, but the reduction word lives in a static device array of the library (256 bytes
 * per GPU, held until the process ends) instead of a buffer of the context, so the call
 * makes no hipMalloc, hipFree or other allocating call.  n is limited to [1, 2^31) as for
 * treepm_timestep (ERR_ARG beyond); the scratch does not grow with n.  Every call on one GPU
 * shares the array and clears it itself (a fill kernel, not hipMemset); calls that overlap
 * on one GPU race and must be serialised by the caller.  ERR_DEVICE if the array's device
 * address cannot be obtained.  Synchronises with the stream's work. */
int treepm_timestep_noalloc(treepm_ctx *ctx, int64_t n, const double *vx, const double *vy,
                            const double *vz, const void *ax, const void *ay, const void *az,
                            int acc_prec, double eps, double zeta, void *hip_stream,
                            double *dt);

/* One kick and drift, in place: v += a dt_kick, then x += v dt_drift, and each coordinate is
 * wrapped back into [0, L) by one box length (one that rounds to L is set to 0).  A leapfrog
 * starts with dt_kick = dt / 2.  Stream-ordered; does not synchronise. */
int treepm_kick_drift(treepm_ctx *ctx, int64_t n, double *x, double *y, double *z, double *vx,
                      double *vy, double *vz, const void *ax, const void *ay, const void *az,
                      int acc_prec, double dt_kick, double dt_drift, void *hip_stream);

/* Choose n_crit (Section 3.1.2's N_crit) for this box by measurement: for each of the
 * n_candidates values (1..64 of them, each >= 1), build, walk and run the FP32 force twice on
 * the given particles (same arguments as treepm_build) and time the second run with device
 * events; the fastest is kept.  Afterwards the context's n_crit is the winner (*best; its
 * time in ms in *best_ms, either may be NULL) and the box is built and walked with it.  Uses
 * the context's other parameters and the FP32 kernel for the trials. */
int treepm_autotune(treepm_ctx *ctx, int64_t n, const double *x, const double *y,
                    const double *z, const double *m, int mem_kind, void *hip_stream,
                    const int32_t *candidates, int32_t n_candidates, int32_t *best,
                    double *best_ms);

/* Counts (and timings) of the last calls.  Synchronises the context's last stream. */
int treepm_get_stats(treepm_ctx *ctx, treepm_stats *stats);

/* ------------------------------------------------------------ exports (host buffers) */

/* Sorted Morton keys and, for each sorted particle, its input index (n each). */
int treepm_export_sorted(treepm_ctx *ctx, uint64_t *keys, int64_t *idx);

/* Tree nodes (cap >= n_nodes): code = (1 << 3 level) | key prefix, first and count in key
 * order, number of children, FP64 mass and centre of mass (com: 3 doubles per node). */
int treepm_export_nodes(treepm_ctx *ctx, int64_t cap, uint64_t *code, int64_t *first,
                        int64_t *count, int32_t *nchild, double *mass, double *com);

/* Groups in key order (cap >= n_groups): node code, first, count, bounding box lo/hi and
 * cube centre x_g (3 doubles each per group). */
int treepm_export_groups(treepm_ctx *ctx, int64_t cap, uint64_t *code, int64_t *first,
                         int64_t *count, double *lo, double *hi, double *xg);

/* Interaction lists in canonical form: offsets[n_groups + 1] (groups in key order); for each
 * entry is_cell (1 = tree node, 0 = particle) and value = node code or the particle's input
 * index.  Entries of one group are in the library's traversal order.  entry_cap must be >=
 * the number of entries (ERR_ARG otherwise). */
int treepm_export_lists(treepm_ctx *ctx, int64_t group_cap, int64_t entry_cap, int64_t *offsets,
                        uint8_t *is_cell, uint64_t *value);

/* The FP32 pair routine of treepm_force_short on explicit positions, pair by pair (the
 * pairwise-accuracy measurement of Section 3.1.1): out[(i n_j + j) 3 + a] is the
 * acceleration at xi[i] from a mass mj[j] at xj[j], computed exactly as the force kernel
 * does -- coordinates relative to xg and in units of r_cut, FP32 arithmetic and the box's
 * table of the pair law -- but without periodic images and without the cull of sources
 * beyond r_cut.
 * xi: 3 n_i doubles, xj: 3 n_j, mj: n_j, xg: 3, out: 3 n_i n_j (all host memory).
 * n_i n_j <= 2^28.  Uses params->r_cut and params->eps (validated as for treepm_create). */
int treepm_pairwise_f32(const treepm_params *params, int device, int64_t n_i, const double *xi,
                        int64_t n_j, const double *xj, const double *mj, const double *xg,
                        double *out);

/* ------------------------------------------------------------ ensemble serving */

/* Create a server for force evaluations on many independent boxes on device `device`.
 * hbm_budget: device bytes the server may keep allocated for resident boxes (particles,
 * tree, lists; > 0).  max_inflight: requests run at once (1..16), each on its own worker
 * thread and HIP stream.  A box (identified by the caller's box_id) keeps its device state
 * between requests until it is evicted, least recently used first, to admit another box.
 * An evicted box's device memory stays with the library for the next boxes (treepm_destroy),
 * so the process can hold up to a quarter of the device's memory beyond the budget. */
int treepm_ens_create(int device, size_t hbm_budget, int max_inflight, treepm_ens **out);

/* Shared launches in the server (enable = 1; 0, the default, switches them off).  When on, a
 * worker that has built a box hands it to a ready list instead of walking it, and whenever no
 * batch is running the next free worker takes every ready box (up to 16) and runs their walks
 * and forces with treepm_force_short_batch (Section 2.2 steps 5 and 6 for all of them in one
 * traversal launch and one force launch per size class) while the other workers build the
 * next boxes.  Results are those of the boxes alone, bit for bit.  Takes effect for boxes
 * built after the call.  ERR_ARG for a NULL server or another value of enable. */
int treepm_ens_set_batching(treepm_ens *ens, int enable);

/* Stop the server: queued requests are dropped, running ones finish, all device memory is
 * released.  NULL is accepted. */
int treepm_ens_destroy(treepm_ens *ens);

/* Queue one FP32 force evaluation of box `box_id` with n particles (host arrays, copied
 * before return; same requirements as treepm_build; params->precision must be FP32).
 * Thread-safe.  *ticket identifies the request.  ERR_ARG for invalid input, ERR_OOM if the
 * box alone cannot fit in the budget, ERR_QUEUE_FULL if 4096 requests are queued.  Range
 * errors in the positions are reported by poll. */
int treepm_ensemble_submit(treepm_ens *ens, uint64_t box_id, const treepm_params *params,
                           int64_t n, const double *x, const double *y, const double *z,
                           const double *m, uint64_t *ticket);

/* Non-blocking: TREEPM_PENDING while the request is queued or running; TREEPM_OK when done,
 * after copying the n accelerations of each axis (caller's original order, float) into
 * ax, ay, az (host; NULL skips an axis) and the request's counts and latency into *stats
 * (NULL allowed).  A finished ticket is released by this call (a second poll gives ERR_ARG);
 * a failed request returns its error code once.  Thread-safe. */
int treepm_ensemble_poll(treepm_ens *ens, uint64_t ticket, float *ax, float *ay, float *az,
                         treepm_stats *stats);

/* Snapshot of the server: queued and running requests, resident bytes and boxes. */
int treepm_ens_info(treepm_ens *ens, int64_t *queued, int64_t *inflight,
                    int64_t *resident_bytes, int64_t *resident_boxes);

/* Text of the last error on this context ("" if none).  Valid until the next call. */
const char *treepm_last_error(const treepm_ctx *ctx);

/* Library version string. */
const char *treepm_version(void);

#ifdef __cplusplus
}
#endif

#endif /* TREEPM_H */
