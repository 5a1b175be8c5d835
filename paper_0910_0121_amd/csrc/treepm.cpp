// C ABI of the short-range TreePM tree force: context management, argument checks, device
// buffers, and the order of the kernels of one build / walk / force evaluation.
#include "treepm.h"

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "common.hpp"

#define TREEPM_API extern "C" __attribute__((visibility("default")))

using namespace tpm;

namespace {

struct Buf {
    void *p = nullptr;
    size_t bytes = 0;
    template <typename T>
    T *as() const
    {
        return static_cast<T *>(p);
    }
};

constexpr int kDefaultNCrit = 128;

} // namespace

struct treepm_ctx {
    treepm_params prm{};
    int device = 0;
    // A private stream: destroying the context releases its buffers in a call scope on it,
    // after the context's own work has finished.
    hipStream_t own = nullptr;
    // Recorded on the call's stream as each API call returns: all of this context's work is
    // before it, so destroying the context waits for it rather than for its last stream,
    // which other work (another context's, in a serving worker) may share.
    hipEvent_t idle = nullptr;
    bool idle_set = false;
    hipStream_t cur = nullptr;
    // The FP32 force's size classes run concurrently on the call's stream and these.
    static constexpr int kSubStreams = 3;
    hipStream_t sub[kSubStreams] = {};
    hipEvent_t fork = nullptr, join[kSubStreams] = {};
    std::string err;
    int state = 0; // 0 empty, 1 built, 2 walked
    int64_t n = 0;
    hipStream_t last = nullptr;
    bool timing = false;
    hipEvent_t ev[6] = {};
    bool ev_valid[3] = {false, false, false};
    // particles and sort
    Buf in[4], key, key_alt, idx, idx_alt, hist, scan32, flags, levcnt, gstart, gflag;
    // Per particle in input order, 32 bytes: the build's (x, y, z, m) records for the gather;
    // after the build, the force's acceleration records (float4 or double4).
    Buf rec;
    // nodes
    Buf n_code, n_first, n_count, n_cf, n_parent, n_nch, n_level, n_mass, n_com[3], n_cn[3];
    Buf n_walk; // packed per-node walk records
    Buf tree_sl, tree_blk; // flat octree build: per-particle levels, per-block level counts
    Buf n_src;  // per-node (com, mass) records
    Buf psrc;   // key-ordered particle (x, y, z, m) records
    size_t node_cap = 0;
    uint32_t n_nodes = 0;
    std::vector<uint32_t> lvl;
    int max_level = 0;
    // groups
    Buf g_node, g_first, g_count, g_cg[3], g_hg[3], g_xg[3], g_lo[3], g_hi[3], g_misc;
    size_t group_cap = 0;
    uint32_t n_groups = 0;
    unsigned min_group_level = 0, max_group = 0;
    // lists
    Buf off, glen, wctr, scan64, entries, wstats, overflow, gcells, cls, kept, kept_sum, out[3], bnd, runs;
    int last_force_prec = -1;
    uint32_t class_counts[kForceClasses] = {};
    uint64_t n_entries = 0;
    // From the last walk on this context: total list entries, the longest list and the number
    // of groups, used to size the one-pass walk's pool (0: no walk yet, use two passes).
    uint64_t walk_hint = 0, walk_hint_max = 0;
    // Host-mapped words that kernels publish small results into (see fetch); null if the
    // allocation failed, and then results are copied with a stream synchronisation.
    uint32_t *mbox_h = nullptr, *mbox_d = nullptr;
    uint32_t mseq = 0;
    uint32_t walk_hint_groups = 0;
    int walk_passes = TREEPM_WALK_AUTO; // treepm_set_walk_passes
    uint64_t st[3] = {0, 0, 0};
    // FP32 pair-law table: device copy, and the eps / eta it was built for (0: none)
    Buf tab;
    double tab_key = 0.0;
    ForceTable ftab{};
    int n_cu = 256; // compute units of the device (persistent force grids)
    // particle mesh: fixed-point masses (later the potential), the complex work mesh, the
    // force mesh, the Green's table, twiddles, max mass
    Buf pm_mass, pm_grid, pm_f, pm_green, pm_tw, pm_mx;
    // mass assignment scratch: per mesh cell first particle and chunk offsets, the chunks'
    // boxes of partial sums
    Buf pm_cells, pm_slots;
    // per particle: the mesh force in the caller's order (x, y, z, 0)
    Buf pm_stage;
    Buf n_q; // per node second moment (6 doubles), quadrupole boxes only
    Buf bdesc; // shared launches led by this context: the boxes' descriptors and counters
    Buf step_min; // time-step reduction result
    int pm_n = 0; // mesh size, box and eta the table was built for
    double pm_L = 0.0, pm_eta = 0.0;
};

namespace {

int fail(treepm_ctx *c, int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c) c->err = buf;
    return code;
}

int hip_fail(treepm_ctx *c, hipError_t e, const char *what)
{
    int code = (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) ? TREEPM_ERR_OOM
                                                                           : TREEPM_ERR_DEVICE;
    return fail(c, code, "%s: %s", what, hipGetErrorString(e));
}

#define HIPCHK(ctx, call)                                                                      \
    do {                                                                                       \
        hipError_t e_ = (call);                                                                \
        if (e_ != hipSuccess) return hip_fail((ctx), e_, #call);                               \
    } while (0)

// The context whose buffers reserve()/release() manage on this thread (set by each call).
thread_local treepm_ctx *t_ctx = nullptr;

// ------------------------------------------------------------------ device memory
// Released device buffers are kept, per device, for the next buffers of any context instead
// of going back to the driver: a server that evicts and creates boxes all the time would
// otherwise hand gigabytes a second back and forth, and freeing and mapping device memory
// holds up the other streams' HIP calls meanwhile.  A block released while work on a stream
// may still use it carries an event recorded on that stream and is taken again only once the
// event has completed.  What is kept is bounded (a quarter of the device's memory): past
// that, completed blocks go back to the driver, largest first; an allocation that fails gives
// back everything kept on the device and tries once more.  treepm_release_cached empties it.
struct Block {
    void *p = nullptr;
    size_t bytes = 0;
    hipEvent_t done = nullptr; // recorded where the last work that may use it was queued
};

struct DevCache {
    std::mutex mu;
    std::multimap<size_t, Block> blocks; // by size
    std::vector<hipEvent_t> spare;       // events of blocks taken again
    size_t kept = 0, cap = 0;
};

DevCache g_dev[kMaxDevices];

// Sizes of fresh blocks: powers of two up to 1 MiB, then multiples of 2 MiB, so that a block
// serves later requests of nearby sizes.
size_t block_size(size_t bytes)
{
    if (bytes <= ((size_t)1 << 20)) {
        size_t b = 4096;
        while (b < bytes) b <<= 1;
        return b;
    }
    const size_t g = (size_t)2 << 20;
    return (bytes + g - 1) / g * g;
}

// With d.mu held: has the block's last use completed?  Queried only while this thread holds
// no unread HIP error, which the query's not-ready status would otherwise replace.
bool block_ready(DevCache &d, Block &b, bool may_query)
{
    if (!b.done) return true;
    if (!may_query) return false;
    const hipError_t e = hipEventQuery(b.done);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    d.spare.push_back(b.done);
    b.done = nullptr;
    return true;
}

// With d.mu held: give completed blocks back to the driver, largest first, until at most
// `keep` bytes are kept (with wait, blocks still in use are waited for and given back too).
void trim_blocks(DevCache &d, size_t keep, bool wait)
{
    const bool may_query = hipPeekAtLastError() == hipSuccess;
    for (auto it = d.blocks.end(); it != d.blocks.begin() && d.kept > keep;) {
        --it;
        Block &b = it->second;
        if (wait && b.done) {
            (void)hipEventSynchronize(b.done);
            d.spare.push_back(b.done);
            b.done = nullptr;
        }
        if (!block_ready(d, b, may_query)) continue;
        (void)hipFree(b.p);
        d.kept -= b.bytes;
        it = d.blocks.erase(it);
    }
}

// A block of at least `bytes` on the current device (*got: its size), or an error.
hipError_t take_block(int device, size_t bytes, void **p, size_t *got)
{
    DevCache &d = g_dev[device];
    {
        std::lock_guard<std::mutex> lk(d.mu);
        const bool may_query = hipPeekAtLastError() == hipSuccess;
        // the smallest completed block that holds the request
        // (at most half again its size)
        const size_t hi = bytes <= ((size_t)1 << 20) ? ((size_t)1 << 20) : bytes + bytes / 2;
        for (auto it = d.blocks.lower_bound(bytes); it != d.blocks.end() && it->first <= hi;
             ++it)
            if (block_ready(d, it->second, may_query)) {
                *p = it->second.p;
                *got = it->second.bytes;
                d.kept -= it->second.bytes;
                d.blocks.erase(it);
                return hipSuccess;
            }
    }
    const size_t want = block_size(bytes);
    hipError_t e = hipMalloc(p, want);
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) {
        (void)hipGetLastError();
        {
            std::lock_guard<std::mutex> lk(d.mu);
            trim_blocks(d, 0, true);
        }
        e = hipMalloc(p, want);
    }
    if (e != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        return e;
    }
    *got = want;
    return hipSuccess;
}

// Keep a block for reuse; `in_use` (may be null) is a stream whose queued work may still use
// it.
void give_block(int device, void *p, size_t bytes, hipStream_t in_use, bool pending)
{
    DevCache &d = g_dev[device];
    std::lock_guard<std::mutex> lk(d.mu);
    if (!d.cap) {
        size_t fr = 0, tot = 0;
        d.cap = hipMemGetInfo(&fr, &tot) == hipSuccess ? tot / 4 : ((size_t)16 << 30);
        (void)hipGetLastError();
    }
    Block b;
    b.p = p;
    b.bytes = bytes;
    if (pending) {
        hipEvent_t ev = nullptr;
        if (!d.spare.empty()) {
            ev = d.spare.back();
            d.spare.pop_back();
        } else if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
            ev = nullptr;
        }
        if (!ev || hipEventRecord(ev, in_use) != hipSuccess) {
            // no event: wait here for the stream instead
            if (ev) d.spare.push_back(ev);
            ev = nullptr;
            (void)hipStreamSynchronize(in_use);
        }
        b.done = ev;
    }
    d.blocks.emplace(bytes, b);
    d.kept += bytes;
    if (d.kept > d.cap) trim_blocks(d, d.cap, false);
}

void release(Buf &b)
{
    if (!b.p) return;
    treepm_ctx *c = t_ctx;
    if (c && c->device < kMaxDevices) {
        // work queued on the current call's stream may still use the buffer; in the private
        // stream's scope (destroy) the context's work has finished
        give_block(c->device, b.p, b.bytes, c->cur, c->cur != c->own || !c->own);
    } else {
        (void)hipFree(b.p);
    }
    b.p = nullptr;
    b.bytes = 0;
}

hipError_t reserve(Buf &b, size_t bytes)
{
    if (bytes <= b.bytes && b.p) return hipSuccess;
    release(b);
    size_t want = bytes + bytes / 8 + 256;
    treepm_ctx *c = t_ctx;
    hipError_t e;
    size_t got = 0;
    if (c && c->device < kMaxDevices) {
        e = take_block(c->device, want, &b.p, &got);
    } else {
        e = hipMalloc(&b.p, want);
        got = want;
    }
    if (e != hipSuccess) {
        b.p = nullptr;
        b.bytes = 0;
        (void)hipGetLastError();
        return e;
    }
    b.bytes = got;
    return hipSuccess;
}

// Enter an API call on context c with stream s: allocation bookkeeping follows s.
struct CallScope {
    treepm_ctx *prev, *ctx;
    hipStream_t stream;
    CallScope(treepm_ctx *c, hipStream_t s) : prev(t_ctx), ctx(c), stream(s)
    {
        t_ctx = c;
        if (c) c->cur = s;
    }
    ~CallScope()
    {
        if (ctx && ctx->idle && hipEventRecord(ctx->idle, stream) == hipSuccess)
            ctx->idle_set = true;
        t_ctx = prev;
    }
};

int check_params(treepm_ctx *c, const treepm_params *p)
{
    if (!p) return fail(c, TREEPM_ERR_ARG, "params is NULL");
    if (!std::isfinite(p->L) || !(p->L > 0.0)) return fail(c, TREEPM_ERR_ARG, "L must be > 0");
    if (!std::isfinite(p->mesh) || !(p->mesh > 0.0))
        return fail(c, TREEPM_ERR_ARG, "mesh must be > 0");
    if (!std::isfinite(p->r_cut) || !(p->r_cut > 0.0) || p->r_cut > 0.5 * p->L)
        return fail(c, TREEPM_ERR_ARG, "r_cut must satisfy 0 < r_cut <= L/2");
    if (std::fabs(p->r_cut - 3.0 * p->mesh) > 1e-12 * p->r_cut)
        return fail(c, TREEPM_ERR_ARG, "r_cut must equal 3 * mesh (2 eta = r_cut = 3 / N_PM)");
    if (!std::isfinite(p->eps) || p->eps < 0.0) return fail(c, TREEPM_ERR_ARG, "eps must be >= 0");
    if (!std::isfinite(p->theta) || p->theta < 0.0 || p->theta > 1.0)
        return fail(c, TREEPM_ERR_ARG, "theta must be in [0, 1]");
    if (p->opening != TREEPM_OPEN_FIXED && p->opening != TREEPM_OPEN_DISTANCE)
        return fail(c, TREEPM_ERR_ARG, "opening must be TREEPM_OPEN_FIXED or _DISTANCE");
    if (p->opening == TREEPM_OPEN_DISTANCE &&
        (!std::isfinite(p->theta_max) || p->theta_max < 0.0 || p->theta_max > 1.0))
        return fail(c, TREEPM_ERR_ARG, "theta_max must be in [0, 1]");
    if (p->quadrupole != 0 && p->quadrupole != 1)
        return fail(c, TREEPM_ERR_ARG, "quadrupole must be 0 or 1");
    if (p->n_leaf < 2) return fail(c, TREEPM_ERR_ARG, "n_leaf must be >= 2");
    if (p->n_crit < 0) return fail(c, TREEPM_ERR_ARG, "n_crit must be >= 1 (0 = default)");
    if (p->precision != TREEPM_FP32 && p->precision != TREEPM_FP64)
        return fail(c, TREEPM_ERR_ARG, "precision must be TREEPM_FP32 or TREEPM_FP64");
    if (p->precision == TREEPM_FP32 && !(p->eps > 0.0))
        return fail(c, TREEPM_ERR_ARG, "the FP32 kernel requires eps > 0");
    if (p->precision == TREEPM_FP32 && !(p->eps >= std::ldexp(0.5 * p->r_cut, -12)))
        return fail(c, TREEPM_ERR_ARG,
                    "the FP32 kernel's pair-law table needs eps >= 2^-12 r_cut / 2; use "
                    "TREEPM_FP64");
    return TREEPM_OK;
}

NodeArrays nodes_view(treepm_ctx *c)
{
    NodeArrays nd;
    nd.code = c->n_code.as<uint64_t>();
    nd.first = c->n_first.as<uint32_t>();
    nd.count = c->n_count.as<uint32_t>();
    nd.child_first = c->n_cf.as<uint32_t>();
    nd.parent = c->n_parent.as<uint32_t>();
    nd.nchild = c->n_nch.as<uint8_t>();
    nd.level = c->n_level.as<uint8_t>();
    nd.mass = c->n_mass.as<double>();
    nd.comx = c->n_com[0].as<double>();
    nd.comy = c->n_com[1].as<double>();
    nd.comz = c->n_com[2].as<double>();
    nd.cnx = c->n_cn[0].as<double>();
    nd.cny = c->n_cn[1].as<double>();
    nd.cnz = c->n_cn[2].as<double>();
    nd.nsrc = c->n_src.as<double4>();
    nd.psrc = c->psrc.as<double4>();
    return nd;
}

GroupArrays groups_view(treepm_ctx *c)
{
    GroupArrays g;
    g.node = c->g_node.as<uint32_t>();
    g.first = c->g_first.as<uint32_t>();
    g.count = c->g_count.as<uint32_t>();
    g.cgx = c->g_cg[0].as<double>(); g.cgy = c->g_cg[1].as<double>(); g.cgz = c->g_cg[2].as<double>();
    g.hgx = c->g_hg[0].as<double>(); g.hgy = c->g_hg[1].as<double>(); g.hgz = c->g_hg[2].as<double>();
    g.xgx = c->g_xg[0].as<double>(); g.xgy = c->g_xg[1].as<double>(); g.xgz = c->g_xg[2].as<double>();
    g.lox = c->g_lo[0].as<double>(); g.loy = c->g_lo[1].as<double>(); g.loz = c->g_lo[2].as<double>();
    g.hix = c->g_hi[0].as<double>(); g.hiy = c->g_hi[1].as<double>(); g.hiz = c->g_hi[2].as<double>();
    return g;
}

// Node arrays with room for `need` nodes; existing contents (n_nodes) are kept.
int ensure_nodes(treepm_ctx *c, size_t need, hipStream_t s)
{
    if (need <= c->node_cap) return TREEPM_OK;
    size_t cap = std::max(need, c->node_cap * 2);
    struct F {
        Buf *b;
        size_t elem;
    } fields[] = {{&c->n_code, 8}, {&c->n_first, 4}, {&c->n_count, 4}, {&c->n_cf, 4},
                  {&c->n_parent, 4}, {&c->n_nch, 1}, {&c->n_level, 1}, {&c->n_mass, 8},
                  {&c->n_com[0], 8}, {&c->n_com[1], 8}, {&c->n_com[2], 8}, {&c->n_cn[0], 8},
                  {&c->n_cn[1], 8}, {&c->n_cn[2], 8}};
    for (auto &f : fields) {
        Buf nb;
        hipError_t e = reserve(nb, cap * f.elem);
        if (e != hipSuccess) return hip_fail(c, e, "node arrays");
        if (f.b->p && c->n_nodes) {
            e = hipMemcpyAsync(nb.p, f.b->p, (size_t)c->n_nodes * f.elem,
                               hipMemcpyDeviceToDevice, s);
            if (e != hipSuccess) return hip_fail(c, e, "node copy");
        }
        release(*f.b); // stream-ordered after the copy
        *f.b = nb;
    }
    c->node_cap = cap;
    return TREEPM_OK;
}

// The walk records and source records of c->n_nodes nodes (written by the moments pass).
int reserve_node_records(treepm_ctx *c)
{
    hipError_t e = reserve(c->n_walk, (size_t)c->n_nodes * sizeof(WalkNode));
    if (e == hipSuccess) e = reserve(c->n_src, (size_t)c->n_nodes * sizeof(double4));
    if (e != hipSuccess) return hip_fail(c, e, "walk records");
    return TREEPM_OK;
}

int ensure_groups(treepm_ctx *c, size_t need)
{
    if (need <= c->group_cap && c->g_node.p) return TREEPM_OK;
    size_t cap = need + need / 8 + 64;
    Buf *u32s[] = {&c->g_node, &c->g_first, &c->g_count};
    for (Buf *b : u32s) {
        hipError_t e = reserve(*b, cap * 4);
        if (e != hipSuccess) return hip_fail(c, e, "group arrays");
    }
    Buf *f64s[] = {&c->g_cg[0], &c->g_cg[1], &c->g_cg[2], &c->g_hg[0], &c->g_hg[1], &c->g_hg[2],
                   &c->g_xg[0], &c->g_xg[1], &c->g_xg[2], &c->g_lo[0], &c->g_lo[1], &c->g_lo[2],
                   &c->g_hi[0], &c->g_hi[1], &c->g_hi[2]};
    for (Buf *b : f64s) {
        hipError_t e = reserve(*b, cap * 8);
        if (e != hipSuccess) return hip_fail(c, e, "group arrays");
    }
    c->group_cap = cap;
    return TREEPM_OK;
}

template <typename T>
int d2h(treepm_ctx *c, T *dst, const void *src, size_t count, hipStream_t s)
{
    if (!count) return TREEPM_OK;
    HIPCHK(c, hipMemcpyAsync(dst, src, count * sizeof(T), hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    return TREEPM_OK;
}

// Mailboxes come from slabs of pinned, mapped, coherent host memory that are kept for the
// life of the process: contexts are created and destroyed often (the ensemble evicts boxes),
// and pinning or unpinning host memory would stall every stream on the device.
std::mutex g_mbox_mu;
std::vector<std::pair<uint32_t *, uint32_t *>> g_mbox_free; // (host, device)

void take_mailbox(uint32_t **h, uint32_t **d)
{
    std::lock_guard<std::mutex> lk(g_mbox_mu);
    *h = *d = nullptr;
    if (g_mbox_free.empty()) {
        constexpr int kSlab = 64;
        uint32_t *hp = nullptr, *dp = nullptr;
        if (hipHostMalloc((void **)&hp, (size_t)kSlab * kMailboxWords * 4,
                          hipHostMallocMapped | hipHostMallocCoherent |
                              hipHostMallocPortable) != hipSuccess ||
            hipHostGetDevicePointer((void **)&dp, hp, 0) != hipSuccess) {
            (void)hipGetLastError();
            return; // the caller copies instead
        }
        for (int i = 0; i < kSlab; ++i)
            g_mbox_free.emplace_back(hp + (size_t)i * kMailboxWords, dp + (size_t)i * kMailboxWords);
    }
    *h = g_mbox_free.back().first;
    *d = g_mbox_free.back().second;
    g_mbox_free.pop_back();
    std::memset(*h, 0, kMailboxWords * 4); // no sequence number of a former owner survives
}

void give_mailbox(uint32_t *h, uint32_t *d)
{
    std::lock_guard<std::mutex> lk(g_mbox_mu);
    g_mbox_free.emplace_back(h, d);
}

// Small device results to the host: up to three runs of 4-byte-multiple objects, published
// by one kernel into the mapped mailbox, waited for by spinning on its sequence word (with
// the stream's state checked, so a failed stream ends the wait).  Falls back to d2h.
struct Run3 {
    void *dst;
    const void *src;
    size_t bytes;
};

// fetch in two halves, so that several contexts' results can be queued before the host
// waits: fetch_post queues the publishing kernel (or, without a mailbox or for too many words,
// copies at once) and returns the sequence number to wait for (0: already copied).
int fetch_post(treepm_ctx *c, hipStream_t s, uint32_t *seq_out, Run3 a,
               Run3 b = {nullptr, nullptr, 0}, Run3 d = {nullptr, nullptr, 0})
{
    *seq_out = 0;
    const size_t words = (a.bytes + b.bytes + d.bytes) / 4;
    if (!c->mbox_h || words >= kMailboxWords) {
        int rc;
        for (const Run3 &r : {a, b, d})
            if (r.bytes && (rc = d2h(c, (uint32_t *)r.dst, r.src, r.bytes / 4, s))) return rc;
        return TREEPM_OK;
    }
    uint32_t seq = ++c->mseq;
    if (seq == 0) seq = ++c->mseq;
    publish_words((const uint32_t *)a.src, (uint32_t)(a.bytes / 4), (const uint32_t *)b.src,
                  (uint32_t)(b.bytes / 4), (const uint32_t *)d.src, (uint32_t)(d.bytes / 4),
                  c->mbox_d, seq, s);
    HIPCHK(c, hipGetLastError());
    *seq_out = seq;
    return TREEPM_OK;
}

int fetch_wait(treepm_ctx *c, hipStream_t s, uint32_t seq, Run3 a,
               Run3 b = {nullptr, nullptr, 0}, Run3 d = {nullptr, nullptr, 0})
{
    if (!seq) return TREEPM_OK;
    for (uint32_t spin = 0;
         __atomic_load_n(&c->mbox_h[0], __ATOMIC_ACQUIRE) != seq; ++spin) {
        if (spin < 2048) {
            __builtin_ia32_pause();
            continue;
        }
        const hipError_t q = hipStreamQuery(s);
        if (q == hipSuccess) {
            if (__atomic_load_n(&c->mbox_h[0], __ATOMIC_ACQUIRE) == seq) break;
            return fail(c, TREEPM_ERR_DEVICE, "a published result did not arrive");
        }
        if (q != hipErrorNotReady) return hip_fail(c, q, "stream");
        std::this_thread::yield();
    }
    const uint32_t *w = c->mbox_h + 1;
    for (const Run3 &r : {a, b, d}) {
        if (r.bytes) std::memcpy(r.dst, w, r.bytes);
        w += r.bytes / 4;
    }
    return TREEPM_OK;
}

int fetch(treepm_ctx *c, hipStream_t s, Run3 a, Run3 b = {nullptr, nullptr, 0},
          Run3 d = {nullptr, nullptr, 0})
{
    uint32_t seq = 0;
    const int rc = fetch_post(c, s, &seq, a, b, d);
    return rc ? rc : fetch_wait(c, s, seq, a, b, d);
}

void record(treepm_ctx *c, int i, hipStream_t s)
{
    if (c->timing) hipEventRecord(c->ev[i], s);
}

int do_build(treepm_ctx *c, int64_t n, const double *x, const double *y, const double *z,
             const double *m, int mem_kind, hipStream_t s)
{
    const treepm_params &P = c->prm;
    int rc;
    size_t N = (size_t)n;
    // particle-sized buffers
    struct R {
        Buf *b;
        size_t bytes;
    } res[] = {{&c->key, N * 8},         {&c->key_alt, N * 8},   {&c->idx, N * 4},
               {&c->idx_alt, N * 4},     {&c->flags, 64},
               {&c->levcnt, (N + 1) * 4 + scan_tmp_elems(N + 1) * 4 + 64},
               {&c->gstart, N * 4},      {&c->gflag, (N + 1) * 4},
               {&c->hist, sort_hist_elems(n) * 4},
               {&c->scan32, (scan_tmp_elems(std::max(sort_hist_elems(n), N + 1)) + 64) * 4},
               {&c->g_misc, 64},
               {&c->rec, N * 32},        {&c->psrc, N * 32}};
    for (auto &r : res) {
        hipError_t e = reserve(*r.b, std::max<size_t>(r.bytes, 64));
        if (e != hipSuccess) return hip_fail(c, e, "particle buffers");
    }
    const double *src[4] = {x, y, z, m};
    if (mem_kind == TREEPM_HOST) {
        for (int a = 0; a < 4; ++a) {
            hipError_t e = reserve(c->in[a], N * 8);
            if (e != hipSuccess) return hip_fail(c, e, "input staging");
            HIPCHK(c, hipMemcpyAsync(c->in[a].p, src[a], N * 8, hipMemcpyHostToDevice, s));
            src[a] = c->in[a].as<double>();
        }
    }
    unsigned *flags = c->flags.as<unsigned>();
    fill_u32(flags, 4, 0u, s);
    launch_keys(n, src[0], src[1], src[2], src[3], P.L, c->key.as<uint64_t>(),
                c->idx.as<uint32_t>(), flags, c->rec.as<double4>(), s);
    uint32_t *scan_tmp = c->scan32.as<uint32_t>();
    {
        // high key bits first, runs of equal high bits sorted in place; all bits if a run is
        // too long for that
        unsigned *sflags = c->flags.as<unsigned>() + 4;
        const uint32_t long_cap = (uint32_t)(N / (kShortRun + 1) + 1);
        hipError_t e = reserve(c->runs, (size_t)long_cap * sizeof(uint2));
        if (e != hipSuccess) return hip_fail(c, e, "sort runs");
        if (radix_sort_high(n, c->key.as<uint64_t>(), c->idx.as<uint32_t>(),
                            c->key_alt.as<uint64_t>(), c->idx_alt.as<uint32_t>(),
                            c->hist.as<uint32_t>(), scan_tmp, c->runs.as<uint2>(), long_cap,
                            sflags, s)) {
            std::swap(c->key, c->key_alt);
            std::swap(c->idx, c->idx_alt);
        }
        // the input checks of k_keys and the sort's fallback flag in one read (sorting
        // invalid input first is harmless: keys are clamped)
        unsigned fl[6] = {};
        if ((rc = fetch(c, s, {fl, flags, sizeof fl}))) return rc;
        if (fl[0] & kFlagNonFinite)
            return fail(c, TREEPM_ERR_ARG, "non-finite position or mass, or a mass <= 0");
        if (fl[0] & kFlagRange)
            return fail(c, TREEPM_ERR_RANGE, "a position lies outside [0, L); wrap it first");
        if (fl[5])
            radix_sort(n, c->key.as<uint64_t>(), c->idx.as<uint32_t>(),
                       c->key_alt.as<uint64_t>(), c->idx_alt.as<uint32_t>(),
                       c->hist.as<uint32_t>(), scan_tmp, s);
    }
    {
        hipError_t e = reserve(c->pm_mx, 8);
        if (e != hipSuccess) return hip_fail(c, e, "largest-mass word");
    }
    // The gather into key order reads only the sort's indices, and the octree passes only the
    // keys: the gather runs on a side stream beside them, and the moments wait for it.
    // Every exit after the fork joins the side stream back into s (an error return too, so
    // nothing is released while the gather may still read it).
    struct SideJoin {
        treepm_ctx *c;
        hipStream_t s, sp;
        ~SideJoin()
        {
            if (sp != s) {
                (void)hipEventRecord(c->join[0], sp);
                (void)hipStreamWaitEvent(s, c->join[0], 0);
            }
        }
    } side{c, s, s};
    if (c->fork) {
        HIPCHK(c, hipEventRecord(c->fork, s));
        HIPCHK(c, hipStreamWaitEvent(c->sub[0], c->fork, 0));
        side.sp = c->sub[0];
    }
    const hipStream_t sp = side.sp;
    launch_permute(n, c->idx.as<uint32_t>(), c->rec.as<double4>(), c->psrc.as<double4>(),
                   c->pm_mx.as<unsigned long long>(), sp);
    // octree: straight from the sorted keys, or level by level for n_leaf above the window
    const double4 *ps = c->psrc.as<double4>();
    uint32_t *cnt = c->levcnt.as<uint32_t>();
    uint32_t *cnt_total = cnt + (N + 1);
    uint32_t *cnt_tmp = cnt_total + 16;
    NodeArrays nd{};
    const bool flat = n >= 1 && P.n_leaf - 1 <= kTreeWin;
    if (flat) {
        const uint32_t nblk = tree_blocks(n);
        hipError_t e = reserve(c->tree_sl, (size_t)n * sizeof(uint32_t));
        if (e == hipSuccess)
            e = reserve(c->tree_blk, ((size_t)nblk * (kMaxLevel + 1) + 64) * sizeof(uint32_t));
        if (e != hipSuccess) return hip_fail(c, e, "tree build buffers");
        uint32_t *blk = c->tree_blk.as<uint32_t>();
        uint32_t *tot = blk + (size_t)nblk * (kMaxLevel + 1);
        launch_tree_levels(c->key.as<uint64_t>(), (uint32_t)n, P.n_leaf,
                           c->tree_sl.as<uint32_t>(), blk, tot, s);
        uint32_t per_level[kMaxLevel + 1] = {};
        if ((rc = fetch(c, s, {per_level, tot, sizeof per_level}))) return rc;
        TreeOffsets to{};
        uint64_t acc = 0;
        c->max_level = 0;
        for (int l = 0; l <= kMaxLevel; ++l) {
            to.off[l] = (uint32_t)acc;
            acc += per_level[l];
            if (per_level[l]) c->max_level = l;
            if (acc > 0x7fffffffull)
                return fail(c, TREEPM_ERR_OVERFLOW, "more than 2^31 tree nodes");
        }
        to.off[kMaxLevel + 1] = to.off[kMaxLevel + 2] = (uint32_t)acc;
        c->n_nodes = 0; // nothing to keep if the arrays grow
        if ((rc = ensure_nodes(c, (size_t)acc, s))) return rc;
        c->n_nodes = (uint32_t)acc;
        c->lvl.assign(to.off, to.off + c->max_level + 2);
        if ((rc = reserve_node_records(c))) return rc;
        nd = nodes_view(c);
        launch_tree_emit(nd, c->key.as<uint64_t>(), c->tree_sl.as<uint32_t>(), blk, to,
                         (uint32_t)n, P.L, s);
    } else {
        c->n_nodes = 0;
        if ((rc = ensure_nodes(c, std::max<size_t>(1024, N / 2 + 64), s))) return rc;
        nd = nodes_view(c);
        launch_root(nd, (uint32_t)n, P.L, s);
        c->n_nodes = 1;
        c->lvl.assign({0u, 1u});
        c->max_level = 0;
        for (int l = 0; l <= kMaxLevel; ++l) {
            uint32_t lo = c->lvl[l], hi = c->lvl[l + 1];
            nd = nodes_view(c);
            {
                hipError_t e = reserve(c->bnd, (size_t)(hi - lo) * 7 * 4);
                if (e != hipSuccess) return hip_fail(c, e, "octant bounds");
            }
            launch_split(nd, c->key.as<uint64_t>(), lo, hi, l, P.n_leaf, cnt,
                         c->bnd.as<uint32_t>(), s);
            scan_u32(cnt, hi - lo, cnt_total, cnt_tmp, s);
            uint32_t add = 0;
            if ((rc = fetch(c, s, {&add, cnt_total, sizeof add}))) return rc;
            c->max_level = l;
            if (add == 0) break;
            if ((uint64_t)hi + add > 0x7fffffffull)
                return fail(c, TREEPM_ERR_OVERFLOW, "more than 2^31 tree nodes");
            if ((rc = ensure_nodes(c, (size_t)hi + add, s))) return rc;
            nd = nodes_view(c);
            launch_emit(nd, c->bnd.as<uint32_t>(), lo, hi, l, hi, cnt, P.L, s);
            c->lvl.push_back(hi + add);
            c->n_nodes = hi + add;
        }
        if ((rc = reserve_node_records(c))) return rc;
    }
    if (sp != s) {
        side.sp = s; // joined here
        HIPCHK(c, hipEventRecord(c->join[0], sp));
        HIPCHK(c, hipStreamWaitEvent(s, c->join[0], 0));
    }
    // moments from the deepest level up (a flat-built tree has its nchild and internal counts
    // set here; the children of level l end where level l + 2 starts)
    nd = nodes_view(c);
    for (int l = c->max_level; l >= 0; --l) {
        const uint32_t child_end =
            (size_t)l + 2 < c->lvl.size() ? c->lvl[l + 2] : c->n_nodes;
        launch_moments(nd, ps, c->lvl[l], c->lvl[l + 1], flat ? 1 : 0, child_end,
                       c->n_walk.as<WalkNode>(), s);
    }
    if (P.quadrupole) {
        hipError_t e = reserve(c->n_q, (size_t)c->n_nodes * 6 * sizeof(double));
        if (e != hipSuccess) return hip_fail(c, e, "second moments");
        for (int l = c->max_level; l >= 0; --l)
            launch_second_moments(nd, ps, c->lvl[l], c->lvl[l + 1], c->n_q.as<double>(), s);
    }
    // groups in key order
    int n_crit = P.n_crit > 0 ? P.n_crit : kDefaultNCrit;
    uint32_t *gstart = c->gstart.as<uint32_t>(), *gflag = c->gflag.as<uint32_t>();
    launch_group_mark(nd, c->n_nodes, n_crit, gstart, gflag, n, s);
    scan_u32(gflag, N + 1, cnt_total, cnt_tmp, s);
    uint32_t ng = 0;
    if ((rc = fetch(c, s, {&ng, cnt_total, sizeof ng}))) return rc;
    if ((rc = ensure_groups(c, ng))) return rc;
    GroupArrays gr = groups_view(c);
    launch_group_compact(gstart, gflag, n, gr.node, s);
    unsigned *misc = c->g_misc.as<unsigned>();
    fill_u32(misc, 1, 255u, s);
    fill_u32(misc + 1, 1, 0u, s);
    launch_group_bbox(nd, gr, ng, ps, misc, misc + 1, s);
    unsigned hm[2] = {0, 0};
    if ((rc = fetch(c, s, {hm, misc, sizeof hm}))) return rc;
    c->n_groups = ng;
    c->min_group_level = hm[0];
    c->max_group = hm[1];
    HIPCHK(c, hipStreamSynchronize(s));
    return TREEPM_OK;
}

// Waves of the one-pass walk: six per SIMD on 256 compute units (measured on the 256^3 box:
// 2.57 ms against 2.66 with seven, the most that stay resident, and 2.75 with eight; fewer
// groups in flight keep more of their tree nodes in L2), about 16 groups each at least.
uint32_t pool_waves(uint32_t G) { return std::max(1u, std::min(6144u, (G + 15) / 16)); }

// Below this many groups the one-pass walk has fewer waves than fill the device, and the two
// passes (a wave per group each) are faster: measured on clustered boxes with n_crit 256,
// 0.25 against 0.41 ms at 6,800 groups, 0.87 against 0.96 at 60,000, equal at 90,000, and
// 2.34 against 1.87 ms at 153,000.
constexpr uint32_t kOnePassMinGroups = 16 * 6144;

// One box's walk in parts, shared by treepm_walk and the shared launches of several boxes.
struct BoxWalk {
    uint32_t G = 0;
    WalkParams wp{};
    bool pooled = false; // one pass into a pool sized from the box's last walk
    uint64_t pool = 0, chunk = 0, reserve_len = 0;
    uint32_t waves = 0;
};

// Buffers, cleared flags and statistics, the opening parameters, and the one-pass layout
// when the last walk of this context sizes it (its pool is then reserved).
int prepare_walk(treepm_ctx *c, hipStream_t s, BoxWalk &bw)
{
    const uint32_t G = c->n_groups;
    hipError_t e;
    if ((e = reserve(c->off, ((size_t)G + 1) * 8)) != hipSuccess) return hip_fail(c, e, "offsets");
    if ((e = reserve(c->glen, ((size_t)G + 1) * 4)) != hipSuccess) return hip_fail(c, e, "lengths");
    if ((e = reserve(c->wctr, 128)) != hipSuccess) return hip_fail(c, e, "counters");
    if ((e = reserve(c->scan64, (scan_tmp_elems((size_t)G + 1) + 64) * 8)) != hipSuccess)
        return hip_fail(c, e, "scan buffer");
    if ((e = reserve(c->wstats, 64)) != hipSuccess) return hip_fail(c, e, "stats");
    if ((e = reserve(c->overflow, 64)) != hipSuccess) return hip_fail(c, e, "flags");
    if ((e = reserve(c->gcells, ((size_t)G + 1) * 4)) != hipSuccess)
        return hip_fail(c, e, "group stats");
    if ((e = reserve(c->cls, (kClsLists + kForceClasses * ((size_t)G + 1)) * 4)) != hipSuccess)
        return hip_fail(c, e, "group classes");
    fill_u32(c->overflow.as<unsigned>(), 1, 0u, s);
    fill_u64(c->wstats.as<uint64_t>(), 4, 0ull, s);
    const treepm_params &P = c->prm;
    const bool open = P.opening == TREEPM_OPEN_DISTANCE;
    const double th_lo = std::min(P.theta_max, P.theta / std::sqrt(0.46));
    bw.G = G;
    bw.wp = WalkParams{P.L,
                       P.r_cut * P.r_cut,
                       open ? P.theta_max * P.theta_max : P.theta * P.theta,
                       open ? th_lo * th_lo : 0.0,
                       0.5 * P.r_cut,
                       P.theta,
                       P.theta_max,
                       (uint32_t)c->n_nodes,
                       open ? 1u : 0u};
    bw.pooled = false;
    const bool one_pass = c->walk_passes == TREEPM_WALK_ONE_PASS ||
                          (c->walk_passes == TREEPM_WALK_AUTO && G >= kOnePassMinGroups);
    if (c->walk_hint && G && one_pass) {
        // One pass, sized from the last walk: chunks of at least four of the longest list,
        // a group tried in the current chunk if twice the mean list length is left there,
        // and a pool of 25 % more entries than then plus one chunk per wave.
        bw.waves = pool_waves(G);
        bw.chunk = std::max<uint64_t>(4 * c->walk_hint_max, 32768);
        const uint64_t mean = c->walk_hint / std::max<uint32_t>(c->walk_hint_groups, 1);
        bw.reserve_len = std::min<uint64_t>(std::max<uint64_t>(2 * mean, 64), bw.chunk / 4);
        bw.pool = c->walk_hint + c->walk_hint / 4 + (uint64_t)bw.waves * bw.chunk;
        bw.pooled = reserve(c->entries, bw.pool * 4) == hipSuccess;
    }
    return TREEPM_OK;
}

// The lists in two passes: counts, their prefix sum, the lists.
int walk_two_pass(treepm_ctx *c, hipStream_t s, const BoxWalk &bw)
{
    const uint32_t G = bw.G;
    uint64_t *off = c->off.as<uint64_t>(), *tot = c->scan64.as<uint64_t>();
    unsigned *ovf = c->overflow.as<unsigned>();
    const WalkNode *wn = c->n_walk.as<WalkNode>();
    GroupArrays gr = groups_view(c);
    fill_u64(off, (size_t)G + 1, 0ull, s);
    launch_walk_count(wn, gr, G, bw.wp, off, ovf, s);
    scan_u64(off, (size_t)G + 1, tot, tot + 1, s);
    uint64_t total = 0;
    unsigned ov = 0;
    int r = fetch(c, s, {&total, tot, sizeof total}, {&ov, ovf, sizeof ov});
    if (r) return r;
    if (ov)
        return fail(c, TREEPM_ERR_OVERFLOW, ov & 2u ? "walk read a bad node index"
                                                    : "walk stack overflow");
    hipError_t e = reserve(c->entries, std::max<size_t>(total, 1) * 4);
    if (e != hipSuccess) return hip_fail(c, e, "interaction lists");
    launch_walk_emit(wn, gr, G, bw.wp, off, c->glen.as<uint32_t>(), c->entries.as<uint32_t>(),
                     ovf, c->gcells.as<uint32_t>(), s);
    return TREEPM_OK;
}

// Statistics and force classes of the lists, queued with the flags for the host.
struct WalkResults {
    unsigned long long hs[4] = {};
    unsigned hov = 0;
    uint32_t seq = 0;
};

int post_walk_results(treepm_ctx *c, hipStream_t s, WalkResults &wr)
{
    const uint32_t G = c->n_groups;
    GroupArrays gr = groups_view(c);
    uint32_t *len = c->glen.as<uint32_t>(), *cls = c->cls.as<uint32_t>();
    launch_walk_stats(gr, G, len, c->gcells.as<uint32_t>(), c->wstats.as<unsigned long long>(), s);
    launch_classify(gr, G, len, cls, G + 1, s);
    return fetch_post(c, s, &wr.seq, {&wr.hov, c->overflow.p, sizeof wr.hov},
                      {c->class_counts, cls + kClsCounts, sizeof c->class_counts},
                      {wr.hs, c->wstats.p, sizeof wr.hs});
}

int wait_walk_results(treepm_ctx *c, hipStream_t s, WalkResults &wr)
{
    int rc = fetch_wait(c, s, wr.seq, {&wr.hov, c->overflow.p, sizeof wr.hov},
                        {c->class_counts, c->cls.as<uint32_t>() + kClsCounts,
                         sizeof c->class_counts},
                        {wr.hs, c->wstats.p, sizeof wr.hs});
    if (rc) return rc;
    if (wr.hov & 3u)
        return fail(c, TREEPM_ERR_OVERFLOW, wr.hov & 2u ? "walk read a bad node index"
                                                         : "walk stack overflow");
    return TREEPM_OK;
}

// Until the results show complete lists: a pool that was too small (bit 4) means two
// passes, then the statistics again.
int settle_walk(treepm_ctx *c, hipStream_t s, const BoxWalk &bw, WalkResults &wr)
{
    int rc;
    while (wr.hov) {
        fill_u32(c->overflow.as<unsigned>(), 1, 0u, s);
        fill_u64(c->wstats.as<uint64_t>(), 4, 0ull, s);
        if ((rc = walk_two_pass(c, s, bw))) return rc;
        wr = WalkResults{};
        if ((rc = post_walk_results(c, s, wr))) return rc;
        if ((rc = wait_walk_results(c, s, wr))) return rc;
    }
    c->n_entries = wr.hs[0] + wr.hs[1];
    c->walk_hint = c->n_entries;
    c->walk_hint_max = wr.hs[3];
    c->walk_hint_groups = bw.G;
    for (int i = 0; i < 3; ++i) c->st[i] = wr.hs[i];
    return TREEPM_OK;
}

int do_walk(treepm_ctx *c, hipStream_t s)
{
    int rc;
    BoxWalk bw;
    if ((rc = prepare_walk(c, s, bw))) return rc;
    if (bw.pooled)
        launch_walk_pool(c->n_walk.as<WalkNode>(), groups_view(c), bw.G, bw.wp, bw.waves, bw.pool,
                         bw.chunk, bw.reserve_len, c->wctr.as<uint32_t>(), c->off.as<uint64_t>(),
                         c->glen.as<uint32_t>(), c->entries.as<uint32_t>(),
                         c->overflow.as<unsigned>(), c->gcells.as<uint32_t>(), s);
    else if ((rc = walk_two_pass(c, s, bw)))
        return rc;
    WalkResults wr;
    if ((rc = post_walk_results(c, s, wr))) return rc;
    if ((rc = wait_walk_results(c, s, wr))) return rc;
    return settle_walk(c, s, bw, wr);
}

void fill_stats(treepm_ctx *c, treepm_stats *st)
{
    memset(st, 0, sizeof *st);
    st->n = c->n;
    st->n_nodes = c->n_nodes;
    st->n_groups = c->n_groups;
    st->max_level = c->max_level;
    st->max_group = (int32_t)c->max_group;
    if (c->state >= 2) {
        st->n_cell_entries = (int64_t)c->st[0];
        st->n_part_entries = (int64_t)c->st[1];
        st->interactions = (int64_t)c->st[2];
    }
    if (c->timing) {
        float t;
        for (int i = 0; i < 3; ++i) {
            if (c->ev_valid[i] &&
                hipEventElapsedTime(&t, c->ev[2 * i], c->ev[2 * i + 1]) == hipSuccess)
                st->t_ms[i] = t;
        }
        st->t_ms[3] = st->t_ms[0] + st->t_ms[1] + st->t_ms[2];
    }
}

} // namespace

// The parameter checks of treepm_create, without a context or a device (used by the ensemble
// server to validate a request before queueing it).
int treepm_internal_check_params(const treepm_params *p) { return check_params(nullptr, p); }

// Device bytes the context holds (used by the ensemble server's HBM accounting).
size_t treepm_internal_ctx_bytes(const treepm_ctx *c)
{
    const Buf *all[] = {&c->in[0], &c->in[1], &c->in[2], &c->in[3], &c->key, &c->key_alt,
                        &c->idx, &c->idx_alt,
                        &c->hist, &c->scan32, &c->flags, &c->levcnt, &c->gstart, &c->gflag,
                        &c->rec, &c->n_code, &c->n_first, &c->n_count, &c->n_cf, &c->n_parent,
                        &c->n_nch, &c->n_level, &c->n_mass, &c->n_com[0], &c->n_com[1],
                        &c->n_com[2], &c->n_cn[0], &c->n_cn[1], &c->n_cn[2], &c->n_walk,
                        &c->n_src, &c->psrc, &c->tree_sl, &c->tree_blk,
                        &c->g_node, &c->g_first, &c->g_count, &c->g_cg[0], &c->g_cg[1],
                        &c->g_cg[2], &c->g_hg[0], &c->g_hg[1], &c->g_hg[2], &c->g_xg[0],
                        &c->g_xg[1], &c->g_xg[2], &c->g_lo[0], &c->g_lo[1], &c->g_lo[2],
                        &c->g_hi[0], &c->g_hi[1], &c->g_hi[2], &c->g_misc, &c->off, &c->glen, &c->wctr, &c->scan64,
                        &c->entries, &c->wstats, &c->overflow, &c->gcells, &c->cls,
                        &c->kept, &c->kept_sum, &c->out[0], &c->out[1], &c->out[2], &c->bnd, &c->runs,
                        &c->tab};
    size_t t = 0;
    for (const Buf *b : all) t += b->bytes;
    return t;
}

TREEPM_API const char *treepm_version(void) { return "treepm-mi355x 0.1"; }

namespace {

// The streams and events of destroyed contexts, kept for the next contexts on the same device:
// creating and destroying them takes milliseconds, and an ensemble evicts and creates boxes
// all the time.  Only complete sets whose streams are idle are kept, at most kMaxShells.
struct Shell {
    int device = 0;
    hipStream_t own = nullptr, sub[treepm_ctx::kSubStreams] = {};
    hipEvent_t idle = nullptr, fork = nullptr, join[treepm_ctx::kSubStreams] = {};
};
constexpr size_t kMaxShells = 64;
std::mutex g_shell_mu;
std::vector<Shell> g_shells;

bool take_shell(int device, Shell *out)
{
    std::lock_guard<std::mutex> lk(g_shell_mu);
    for (size_t i = g_shells.size(); i-- > 0;)
        if (g_shells[i].device == device) {
            *out = g_shells[i];
            g_shells.erase(g_shells.begin() + (std::ptrdiff_t)i);
            return true;
        }
    return false;
}

bool keep_shell(const Shell &sh)
{
    if (!sh.own || !sh.idle || !sh.fork) return false;
    for (int i = 0; i < treepm_ctx::kSubStreams; ++i)
        if (!sh.sub[i] || !sh.join[i]) return false;
    std::lock_guard<std::mutex> lk(g_shell_mu);
    if (g_shells.size() >= kMaxShells) return false;
    g_shells.push_back(sh);
    return true;
}

} // namespace

TREEPM_API int treepm_create(const treepm_params *params, int device, treepm_ctx **out)
{
    if (!out) return TREEPM_ERR_ARG;
    *out = nullptr;
    int rc = check_params(nullptr, params);
    if (rc) return rc;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
        return TREEPM_ERR_DEVICE;
    treepm_ctx *c = new (std::nothrow) treepm_ctx();
    if (!c) return TREEPM_ERR_OOM;
    c->prm = *params;
    c->device = device;
    if (hipSetDevice(device) != hipSuccess) {
        delete c;
        return TREEPM_ERR_DEVICE;
    }
    {
        int ncu = 0;
        if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device) ==
                hipSuccess &&
            ncu > 0)
            c->n_cu = ncu;
        (void)hipGetLastError();
    }
    Shell sh;
    if (take_shell(device, &sh)) {
        c->own = sh.own;
        c->idle = sh.idle;
        c->fork = sh.fork;
        for (int i = 0; i < treepm_ctx::kSubStreams; ++i) {
            c->sub[i] = sh.sub[i];
            c->join[i] = sh.join[i];
        }
        take_mailbox(&c->mbox_h, &c->mbox_d);
        *out = c;
        return TREEPM_OK;
    }
    if (hipStreamCreateWithFlags(&c->own, hipStreamNonBlocking) != hipSuccess) {
        c->own = nullptr; // destroy then releases in the last stream's scope
        (void)hipGetLastError();
    }
    if (hipEventCreateWithFlags(&c->idle, hipEventDisableTiming) != hipSuccess) {
        c->idle = nullptr; // destroy then waits for the last stream instead
        (void)hipGetLastError();
    }
    bool subs_ok = hipEventCreateWithFlags(&c->fork, hipEventDisableTiming) == hipSuccess;
    for (int i = 0; subs_ok && i < treepm_ctx::kSubStreams; ++i)
        subs_ok = hipStreamCreateWithFlags(&c->sub[i], hipStreamNonBlocking) == hipSuccess &&
                  hipEventCreateWithFlags(&c->join[i], hipEventDisableTiming) == hipSuccess;
    if (!subs_ok) { // run the classes one after another on the call's stream
        for (int i = 0; i < treepm_ctx::kSubStreams; ++i) {
            if (c->sub[i]) (void)hipStreamDestroy(c->sub[i]);
            if (c->join[i]) (void)hipEventDestroy(c->join[i]);
            c->sub[i] = nullptr;
            c->join[i] = nullptr;
        }
        if (c->fork) (void)hipEventDestroy(c->fork);
        c->fork = nullptr;
        (void)hipGetLastError();
    }
    // the mailbox for small results (fetch); without it results are copied and synchronised
    take_mailbox(&c->mbox_h, &c->mbox_d);
    *out = c;
    return TREEPM_OK;
}

TREEPM_API int treepm_destroy(treepm_ctx *c)
{
    if (!c) return TREEPM_OK;
    hipSetDevice(c->device);
    // this context's own work, not the rest of a stream it may share
    if (c->idle && c->idle_set) (void)hipEventSynchronize(c->idle);
    else if (c->last) (void)hipStreamSynchronize(c->last);
    else (void)hipDeviceSynchronize();
    hipEvent_t idle = c->idle;
    c->idle = nullptr; // no more records: the scope below must not touch the event
    Buf *all[] = {&c->in[0], &c->in[1], &c->in[2], &c->in[3], &c->key, &c->key_alt, &c->idx,
                  &c->idx_alt, &c->hist,
                  &c->scan32, &c->flags, &c->levcnt, &c->gstart, &c->gflag, &c->n_code,
                  &c->n_first, &c->n_count, &c->n_cf, &c->n_parent, &c->n_nch, &c->n_level,
                  &c->n_mass, &c->n_com[0], &c->n_com[1], &c->n_com[2], &c->n_cn[0],
                  &c->n_cn[1], &c->n_cn[2], &c->n_walk, &c->n_src, &c->psrc, &c->tree_sl,
                  &c->tree_blk, &c->g_node, &c->g_first, &c->g_count, &c->g_cg[0],
                  &c->g_cg[1], &c->g_cg[2], &c->g_hg[0], &c->g_hg[1], &c->g_hg[2], &c->g_xg[0],
                  &c->g_xg[1], &c->g_xg[2], &c->g_lo[0], &c->g_lo[1], &c->g_lo[2], &c->g_hi[0],
                  &c->g_hi[1], &c->g_hi[2], &c->g_misc, &c->off, &c->glen, &c->wctr, &c->scan64, &c->entries,
                  &c->wstats, &c->overflow, &c->rec, &c->kept, &c->kept_sum, &c->gcells, &c->cls, &c->out[0],
                  &c->out[1], &c->out[2], &c->bnd, &c->runs, &c->pm_mass, &c->pm_grid,
                  &c->pm_f, &c->pm_green, &c->pm_tw, &c->pm_mx, &c->pm_stage, &c->pm_cells, &c->pm_slots,
                  &c->n_q, &c->step_min, &c->tab, &c->bdesc};
    {
        // the work is done: the buffers are kept for reuse at once, not behind a stream
        CallScope scope(c, c->own ? c->own : c->last);
        for (Buf *b : all) release(*b);
    }
    if (c->own) (void)hipStreamSynchronize(c->own);
    if (c->mbox_h) give_mailbox(c->mbox_h, c->mbox_d); // the stream is idle: nothing writes it
    Shell sh;
    sh.device = c->device;
    sh.own = c->own;
    sh.idle = idle;
    sh.fork = c->fork;
    for (int i = 0; i < treepm_ctx::kSubStreams; ++i) {
        sh.sub[i] = c->sub[i];
        sh.join[i] = c->join[i];
        if (c->sub[i]) (void)hipStreamSynchronize(c->sub[i]);
    }
    if (!keep_shell(sh)) {
        if (c->own) (void)hipStreamDestroy(c->own);
        if (idle) (void)hipEventDestroy(idle);
        for (int i = 0; i < treepm_ctx::kSubStreams; ++i) {
            if (c->sub[i]) (void)hipStreamDestroy(c->sub[i]);
            if (c->join[i]) (void)hipEventDestroy(c->join[i]);
        }
        if (c->fork) (void)hipEventDestroy(c->fork);
    }
    if (c->ev[0])
        for (hipEvent_t &e : c->ev) (void)hipEventDestroy(e);
    delete c;
    return TREEPM_OK;
}

TREEPM_API int treepm_release_cached(int device)
{
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev ||
        device >= kMaxDevices)
        return TREEPM_ERR_DEVICE;
    if (hipSetDevice(device) != hipSuccess) return TREEPM_ERR_DEVICE;
    DevCache &d = g_dev[device];
    std::lock_guard<std::mutex> lk(d.mu);
    trim_blocks(d, 0, true);
    return TREEPM_OK;
}

TREEPM_API int treepm_set_params(treepm_ctx *c, const treepm_params *params)
{
    if (!c) return TREEPM_ERR_ARG;
    int rc = check_params(c, params);
    if (rc) return rc;
    c->prm = *params;
    c->state = 0;
    return TREEPM_OK;
}

TREEPM_API int treepm_set_walk_passes(treepm_ctx *c, int mode)
{
    if (!c) return TREEPM_ERR_ARG;
    if (mode != TREEPM_WALK_AUTO && mode != TREEPM_WALK_ONE_PASS &&
        mode != TREEPM_WALK_TWO_PASS)
        return fail(c, TREEPM_ERR_ARG, "mode must be TREEPM_WALK_AUTO, _ONE_PASS or _TWO_PASS");
    c->walk_passes = mode;
    return TREEPM_OK;
}

TREEPM_API int treepm_set_timing(treepm_ctx *c, int enable)
{
    if (!c) return TREEPM_ERR_ARG;
    HIPCHK(c, hipSetDevice(c->device));
    if (enable && !c->ev[0])
        for (hipEvent_t &e : c->ev) HIPCHK(c, hipEventCreate(&e));
    c->timing = enable != 0;
    for (bool &v : c->ev_valid) v = false;
    return TREEPM_OK;
}

TREEPM_API int treepm_build(treepm_ctx *c, int64_t n, const double *x, const double *y,
                            const double *z, const double *m, int mem_kind, void *hip_stream)
{
    if (!c) return TREEPM_ERR_ARG;
    c->err.clear();
    c->state = 0;
    if (n < 1 || n > 0x7fffffffLL) return fail(c, TREEPM_ERR_ARG, "n must be in [1, 2^31)");
    if (!x || !y || !z || !m) return fail(c, TREEPM_ERR_ARG, "NULL input buffer");
    if (mem_kind != TREEPM_HOST && mem_kind != TREEPM_DEVICE)
        return fail(c, TREEPM_ERR_ARG, "mem_kind must be TREEPM_HOST or TREEPM_DEVICE");
    HIPCHK(c, hipSetDevice(c->device));
    hipStream_t s = (hipStream_t)hip_stream;
    c->last = s;
    CallScope scope(c, s);
    record(c, 0, s);
    int rc = do_build(c, n, x, y, z, m, mem_kind, s);
    if (rc) return rc;
    record(c, 1, s);
    c->ev_valid[0] = c->timing;
    c->ev_valid[1] = c->ev_valid[2] = false;
    c->n = n;
    c->state = 1;
    return TREEPM_OK;
}

TREEPM_API int treepm_walk(treepm_ctx *c, void *hip_stream, treepm_stats *stats)
{
    if (!c) return TREEPM_ERR_ARG;
    if (c->state < 1) return fail(c, TREEPM_ERR_STATE, "treepm_walk needs a build");
    c->err.clear();
    HIPCHK(c, hipSetDevice(c->device));
    hipStream_t s = (hipStream_t)hip_stream;
    c->last = s;
    CallScope scope(c, s);
    record(c, 2, s);
    int rc = do_walk(c, s);
    if (rc) {
        c->state = 1;
        return rc;
    }
    record(c, 3, s);
    c->ev_valid[1] = c->timing;
    c->state = 2;
    if (stats) fill_stats(c, stats);
    return TREEPM_OK;
}

namespace {

// The FP32 pair-law table of the context's eps / eta, built on the host and copied to the
// device once per parameter set.
int ensure_table(treepm_ctx *c, hipStream_t s)
{
    const double key = c->prm.eps / c->prm.r_cut;
    if (c->tab.p && c->tab_key == key) return TREEPM_OK;
    std::vector<float4> coef;
    uint32_t base = 0;
    float cc = 0.f;
    if (!build_force_table(key, coef, base, cc))
        return fail(c, TREEPM_ERR_ARG, "eps / r_cut = %g is outside the FP32 table's range", key);
    hipError_t e = reserve(c->tab, coef.size() * sizeof(float4));
    if (e != hipSuccess) return hip_fail(c, e, "pair-law table");
    HIPCHK(c, hipMemcpyAsync(c->tab.p, coef.data(), coef.size() * sizeof(float4),
                             hipMemcpyHostToDevice, s));
    HIPCHK(c, hipStreamSynchronize(s)); // coef is a host temporary
    c->ftab = ForceTable{c->tab.as<float4>(), (uint32_t)coef.size(), base, cc};
    c->tab_key = key;
    return TREEPM_OK;
}

} // namespace

namespace {

// The short-range force into ax, ay, az: out mode 0 / 1 stores float / double accelerations,
// 2 (kick) adds kick_dt times them to double velocities.  Arguments checked by the caller.
// The kernels leave one record per particle in c->rec (free once the build has gathered from
// it), which a last pass writes out in the caller's order.
int do_force_short(treepm_ctx *c, void *ax, void *ay, void *az, int out_prec, int mem_kind,
                   void *hip_stream, double kick_dt)
{
    int rc;
    const treepm_params &P = c->prm;
    if (P.precision == TREEPM_FP32) {
        // Positions are taken relative to the group's cube centre with one image per list
        // entry; that image is the nearest one for every particle of the group only if half
        // the group cube plus r_cut stays within L/2.
        double half_side = 0.5 * std::ldexp(P.L, -(int)c->min_group_level);
        if (half_side + P.r_cut > 0.5 * P.L)
            return fail(c, TREEPM_ERR_ARG,
                        "FP32 path needs group cube half-side + r_cut <= L/2 (a group at "
                        "level %u is too large for r_cut); use TREEPM_FP64",
                        c->min_group_level);
    }
    HIPCHK(c, hipSetDevice(c->device));
    hipStream_t s = (hipStream_t)hip_stream;
    c->last = s;
    CallScope scope(c, s);
    size_t esz = out_prec == TREEPM_FP32 ? 4 : 8;
    void *dst[3] = {ax, ay, az};
    if (mem_kind == TREEPM_HOST) {
        for (int a = 0; a < 3; ++a) {
            hipError_t e = reserve(c->out[a], (size_t)c->n * esz);
            if (e != hipSuccess) return hip_fail(c, e, "output staging");
            dst[a] = c->out[a].p;
        }
    }
    record(c, 4, s);
    NodeArrays nd = nodes_view(c);
    GroupArrays gr = groups_view(c);
    double eta = 0.5 * P.r_cut;
    {
        hipError_t e = reserve(c->kept, ((size_t)c->n_groups + 1) * 4);
        if (e == hipSuccess) e = reserve(c->kept_sum, 64);
        if (e != hipSuccess) return hip_fail(c, e, "force statistics");
    }
    ForceParams fp{P.L, P.eps * P.eps, 1.0 / eta, eta, P.r_cut * P.r_cut, P.r_cut,
                   c->kept.as<uint32_t>()};
    const int rec64 = out_prec != TREEPM_FP32;
    void *rec = c->rec.p; // n x 32 bytes since the build
    if (P.precision == TREEPM_FP32) {
        if ((rc = ensure_table(c, s))) return rc;
        hipStream_t streams[1 + treepm_ctx::kSubStreams] = {s};
        int ns = 1;
        launch_force_f32_prep(c->cls.as<uint32_t>(), s); // queues, before the fork
        if (c->fork) {
            HIPCHK(c, hipEventRecord(c->fork, s));
            for (int i = 0; i < treepm_ctx::kSubStreams; ++i) {
                HIPCHK(c, hipStreamWaitEvent(c->sub[i], c->fork, 0));
                streams[ns++] = c->sub[i];
            }
        }
        launch_force_f32(nd, gr, c->cls.as<uint32_t>(), c->class_counts, c->off.as<uint64_t>(),
                         c->glen.as<uint32_t>(), c->entries.as<uint32_t>(),
                         c->psrc.as<double4>(), c->idx.as<uint32_t>(), fp, c->ftab, rec, rec64,
                         c->n_cu, streams, ns);
        if (c->fork)
            for (int i = 0; i < treepm_ctx::kSubStreams; ++i) {
                HIPCHK(c, hipEventRecord(c->join[i], c->sub[i]));
                HIPCHK(c, hipStreamWaitEvent(s, c->join[i], 0));
            }
    } else
        launch_force_f64(nd, gr, c->n_groups, c->off.as<uint64_t>(), c->glen.as<uint32_t>(),
                         c->entries.as<uint32_t>(),
                         c->psrc.as<double4>(), c->idx.as<uint32_t>(), fp, rec, rec64, s);
    if (P.quadrupole)
        launch_quad(nd, gr, c->n_groups, c->off.as<uint64_t>(), c->glen.as<uint32_t>(),
                    c->entries.as<uint32_t>(), c->psrc.as<double4>(), c->idx.as<uint32_t>(),
                    c->n_q.as<double>(), fp, rec, P.precision == TREEPM_FP64, rec64, s);
    launch_force_out(rec, out_prec, (int64_t)c->n, dst[0], dst[1], dst[2], kick_dt, s);
    HIPCHK(c, hipGetLastError());
    record(c, 5, s);
    launch_kept_stats(gr, c->n_groups, c->kept.as<uint32_t>(),
                          c->kept_sum.as<unsigned long long>(), s);
    c->last_force_prec = P.precision;
    c->ev_valid[2] = c->timing;
    if (mem_kind == TREEPM_HOST) {
        void *hdst[3] = {ax, ay, az};
        for (int a = 0; a < 3; ++a)
            HIPCHK(c, hipMemcpyAsync(hdst[a], dst[a], (size_t)c->n * esz, hipMemcpyDeviceToHost,
                                     s));
        HIPCHK(c, hipStreamSynchronize(s));
    }
    return TREEPM_OK;
}

} // namespace

TREEPM_API int treepm_force_short(treepm_ctx *c, void *ax, void *ay, void *az, int out_prec,
                                  int mem_kind, void *hip_stream)
{
    if (!c) return TREEPM_ERR_ARG;
    if (c->state < 2) return fail(c, TREEPM_ERR_STATE, "treepm_force_short needs a walk");
    c->err.clear();
    if (!ax || !ay || !az) return fail(c, TREEPM_ERR_ARG, "NULL output buffer");
    if (out_prec != TREEPM_FP32 && out_prec != TREEPM_FP64)
        return fail(c, TREEPM_ERR_ARG, "out_prec must be TREEPM_FP32 or TREEPM_FP64");
    if (mem_kind != TREEPM_HOST && mem_kind != TREEPM_DEVICE)
        return fail(c, TREEPM_ERR_ARG, "mem_kind must be TREEPM_HOST or TREEPM_DEVICE");
    return do_force_short(c, ax, ay, az, out_prec, mem_kind, hip_stream, 0.0);
}

namespace {

// Binds the buffer bookkeeping (reserve / release) to context c and stream s for a scope.
struct Bind {
    treepm_ctx *prev;
    Bind(treepm_ctx *c, hipStream_t s) : prev(t_ctx)
    {
        t_ctx = c;
        c->cur = s;
    }
    ~Bind() { t_ctx = prev; }
};

// On leaving a batch call every box marks the stream position after its work, as each
// single-box call does (treepm_destroy waits for it).
struct BatchScope {
    treepm_ctx *const *cs;
    int nb;
    hipStream_t s;
    ~BatchScope()
    {
        for (int b = 0; b < nb; ++b) {
            cs[b]->last = s;
            if (cs[b]->idle && hipEventRecord(cs[b]->idle, s) == hipSuccess)
                cs[b]->idle_set = true;
        }
    }
};

// The box descriptors of one shared launch, copied to the leader's device buffer at `at`
// (bytes); the host copy stays alive until the batch has synchronised.
template <typename T>
int upload(treepm_ctx *lead, hipStream_t s, const std::vector<T> &v, size_t at, T **dev)
{
    *dev = reinterpret_cast<T *>(static_cast<char *>(lead->bdesc.p) + at);
    if (!v.empty())
        HIPCHK(lead, hipMemcpyAsync(*dev, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s));
    return TREEPM_OK;
}

WalkBox walk_box(treepm_ctx *c, const BoxWalk &bw, uint32_t g0)
{
    WalkBox w{};
    w.wn = c->n_walk.as<WalkNode>();
    w.gr = groups_view(c);
    w.wp = bw.wp;
    w.off = c->off.as<uint64_t>();
    w.len = c->glen.as<uint32_t>();
    w.entries = c->entries.as<uint32_t>();
    w.gcells = c->gcells.as<uint32_t>();
    w.pool_next = reinterpret_cast<unsigned long long *>(c->wctr.as<uint32_t>() + kXcds);
    w.pool_cap = bw.pool;
    w.chunk = bw.chunk;
    w.reserve = bw.reserve_len;
    w.overflow = c->overflow.as<unsigned>();
    w.g0 = g0;
    w.n_groups = bw.G;
    return w;
}

// The walk of boxes cs[0 .. nb) with shared launches: the boxes whose last walk sizes a pool
// in one pass together, the others in two passes together (one host wait for all their
// list lengths); then every box's statistics and classes, and one wait for all of them.  A
// box whose pool was too small is walked again alone.  Each box ends exactly as treepm_walk
// would leave it.
int batch_walk(treepm_ctx *const *cs, int nb, hipStream_t s)
{
    treepm_ctx *lead = cs[0];
    int rc;
    std::vector<BoxWalk> bw(nb);
    for (int b = 0; b < nb; ++b) {
        Bind bind(cs[b], s);
        if ((rc = prepare_walk(cs[b], s, bw[b]))) return rc;
    }
    std::vector<WalkBox> two, pool;
    std::vector<int> two_ix;
    uint32_t two_total = 0, pool_total = 0, pool_waves_sum = 0;
    for (int b = 0; b < nb; ++b) {
        if (!bw[b].G) continue;
        if (bw[b].pooled) {
            pool.push_back(walk_box(cs[b], bw[b], pool_total));
            pool_total += bw[b].G;
            pool_waves_sum += bw[b].waves;
        } else {
            two.push_back(walk_box(cs[b], bw[b], two_total));
            two_ix.push_back(b);
            two_total += bw[b].G;
        }
    }
    {
        Bind bind(lead, s);
        const size_t bytes = (2 * (size_t)kMaxBatch) * sizeof(WalkBox) +
                             (size_t)kMaxBatch * sizeof(ForceBox) + 256;
        hipError_t e = reserve(lead->bdesc, bytes);
        if (e != hipSuccess) return hip_fail(lead, e, "batch descriptors");
    }
    const size_t at_two = 0, at_pool = (size_t)kMaxBatch * sizeof(WalkBox);
    const size_t at_ctr = 2 * (size_t)kMaxBatch * sizeof(WalkBox) + (size_t)kMaxBatch * sizeof(ForceBox);
    uint32_t *counters = reinterpret_cast<uint32_t *>(static_cast<char *>(lead->bdesc.p) + at_ctr);
    WalkBox *dev = nullptr;
    if (!two.empty()) {
        for (const WalkBox &w : two) fill_u64(w.off, (size_t)w.n_groups + 1, 0ull, s);
        if ((rc = upload(lead, s, two, at_two, &dev))) return rc;
        launch_walk_count_multi(dev, (int)two.size(), two_total, s);
        std::vector<uint64_t> total(two.size());
        std::vector<unsigned> ov(two.size());
        std::vector<uint32_t> seq(two.size());
        for (size_t k = 0; k < two.size(); ++k) {
            treepm_ctx *c = cs[two_ix[k]];
            uint64_t *tot = c->scan64.as<uint64_t>();
            scan_u64(two[k].off, (size_t)two[k].n_groups + 1, tot, tot + 1, s);
            if ((rc = fetch_post(c, s, &seq[k], {&total[k], tot, sizeof total[k]},
                                 {&ov[k], two[k].overflow, sizeof ov[k]})))
                return rc;
        }
        for (size_t k = 0; k < two.size(); ++k) {
            treepm_ctx *c = cs[two_ix[k]];
            if ((rc = fetch_wait(c, s, seq[k], {&total[k], c->scan64.p, sizeof total[k]},
                                 {&ov[k], two[k].overflow, sizeof ov[k]})))
                return rc;
            if (ov[k])
                return fail(c, TREEPM_ERR_OVERFLOW, ov[k] & 2u ? "walk read a bad node index"
                                                               : "walk stack overflow");
            Bind bind(c, s);
            hipError_t e = reserve(c->entries, std::max<size_t>(total[k], 1) * 4);
            if (e != hipSuccess) return hip_fail(c, e, "interaction lists");
            two[k].entries = c->entries.as<uint32_t>();
        }
        if ((rc = upload(lead, s, two, at_two, &dev))) return rc;
        launch_walk_emit_multi(dev, (int)two.size(), two_total, s);
    }
    if (!pool.empty()) {
        for (const WalkBox &w : pool) fill_u64(reinterpret_cast<uint64_t *>(w.pool_next), 1, 0ull, s);
        if ((rc = upload(lead, s, pool, at_pool, &dev))) return rc;
        launch_walk_pool_multi(dev, (int)pool.size(), pool_total,
                               std::max(1u, std::min(8192u, pool_waves_sum)), counters, s);
    }
    std::vector<WalkResults> wr(nb);
    for (int b = 0; b < nb; ++b)
        if ((rc = post_walk_results(cs[b], s, wr[b]))) return rc;
    for (int b = 0; b < nb; ++b)
        if ((rc = wait_walk_results(cs[b], s, wr[b]))) return rc;
    for (int b = 0; b < nb; ++b) {
        Bind bind(cs[b], s);
        if ((rc = settle_walk(cs[b], s, bw[b], wr[b]))) return rc;
    }
    return TREEPM_OK;
}

// The FP32 short-range force of walked boxes with one persistent launch per size class over
// all of them (forked over the leader's sub-streams), then per box the quadrupole terms, the
// float outputs and the statistics; host outputs are copied back and waited for.
int batch_force(treepm_ctx *const *cs, int nb, float *const *ax, float *const *ay,
                float *const *az, int mem_kind, hipStream_t s)
{
    treepm_ctx *lead = cs[0];
    int rc;
    std::vector<ForceBox> fb(nb);
    uint32_t totals[kForceClasses] = {};
    uint32_t max_entries = 0;
    std::vector<std::array<float *, 3>> dst(nb);
    for (int b = 0; b < nb; ++b) {
        treepm_ctx *c = cs[b];
        Bind bind(c, s);
        const treepm_params &P = c->prm;
        if ((rc = ensure_table(c, s))) return rc;
        hipError_t e = reserve(c->kept, ((size_t)c->n_groups + 1) * 4);
        if (e == hipSuccess) e = reserve(c->kept_sum, 64);
        if (e != hipSuccess) return hip_fail(c, e, "force statistics");
        dst[b] = {ax[b], ay[b], az[b]};
        if (mem_kind == TREEPM_HOST)
            for (int a = 0; a < 3; ++a) {
                e = reserve(c->out[a], (size_t)c->n * 4);
                if (e != hipSuccess) return hip_fail(c, e, "output staging");
                dst[b][a] = c->out[a].as<float>();
            }
        const double eta = 0.5 * P.r_cut;
        ForceBox &F = fb[b];
        F.nd = nodes_view(c);
        F.gr = groups_view(c);
        F.cls = c->cls.as<uint32_t>();
        F.off = c->off.as<uint64_t>();
        F.len = c->glen.as<uint32_t>();
        F.entries = c->entries.as<uint32_t>();
        F.ps = c->psrc.as<double4>();
        F.pidx = c->idx.as<uint32_t>();
        F.fp = ForceParams{P.L, P.eps * P.eps, 1.0 / eta, eta, P.r_cut * P.r_cut, P.r_cut,
                           c->kept.as<uint32_t>()};
        F.ft = c->ftab;
        F.rec = c->rec.p;
        uint64_t id;
        std::memcpy(&id, &c->tab_key, sizeof id);
        F.tab_id = id;
        max_entries = std::max(max_entries, c->ftab.entries);
        for (int k = 0; k < kForceClasses; ++k) totals[k] += c->class_counts[k];
        launch_force_f32_prep(F.cls, s);
    }
    ForceBox *dev = nullptr;
    const size_t at_force = 2 * (size_t)kMaxBatch * sizeof(WalkBox);
    if ((rc = upload(lead, s, fb, at_force, &dev))) return rc;
    hipStream_t streams[1 + treepm_ctx::kSubStreams] = {s};
    int ns = 1;
    if (lead->fork) {
        HIPCHK(lead, hipEventRecord(lead->fork, s));
        for (int i = 0; i < treepm_ctx::kSubStreams; ++i) {
            HIPCHK(lead, hipStreamWaitEvent(lead->sub[i], lead->fork, 0));
            streams[ns++] = lead->sub[i];
        }
    }
    launch_force_f32_multi(dev, nb, totals, max_entries, lead->n_cu, streams, ns);
    if (lead->fork)
        for (int i = 0; i < treepm_ctx::kSubStreams; ++i) {
            HIPCHK(lead, hipEventRecord(lead->join[i], lead->sub[i]));
            HIPCHK(lead, hipStreamWaitEvent(s, lead->join[i], 0));
        }
    for (int b = 0; b < nb; ++b) {
        treepm_ctx *c = cs[b];
        const ForceBox &F = fb[b];
        if (c->prm.quadrupole)
            launch_quad(F.nd, F.gr, c->n_groups, F.off, F.len, F.entries, F.ps, F.pidx,
                        c->n_q.as<double>(), F.fp, F.rec, 0, 0, s);
        launch_force_out(F.rec, TREEPM_FP32, (int64_t)c->n, dst[b][0], dst[b][1], dst[b][2],
                         0.0, s);
        launch_kept_stats(F.gr, c->n_groups, c->kept.as<uint32_t>(),
                          c->kept_sum.as<unsigned long long>(), s);
        c->last_force_prec = TREEPM_FP32;
        c->ev_valid[1] = c->ev_valid[2] = false;
    }
    HIPCHK(lead, hipGetLastError());
    if (mem_kind == TREEPM_HOST)
        for (int b = 0; b < nb; ++b) {
            float *hdst[3] = {ax[b], ay[b], az[b]};
            for (int a = 0; a < 3; ++a)
                HIPCHK(cs[b], hipMemcpyAsync(hdst[a], dst[b][a], (size_t)cs[b]->n * 4,
                                             hipMemcpyDeviceToHost, s));
        }
    HIPCHK(lead, hipStreamSynchronize(s)); // the descriptors' host copies may go now
    return TREEPM_OK;
}

} // namespace

TREEPM_API int treepm_force_short_batch(treepm_ctx *const *ctxs, int n_boxes, float *const *ax,
                                        float *const *ay, float *const *az, int mem_kind,
                                        void *hip_stream)
{
    if (!ctxs || n_boxes < 1 || n_boxes > kMaxBatch || !ax || !ay || !az)
        return TREEPM_ERR_ARG;
    for (int b = 0; b < n_boxes; ++b)
        if (!ctxs[b]) return TREEPM_ERR_ARG;
    treepm_ctx *lead = ctxs[0];
    for (int b = 0; b < n_boxes; ++b) {
        treepm_ctx *c = ctxs[b];
        c->err.clear();
        for (int q = 0; q < b; ++q)
            if (ctxs[q] == c) return fail(c, TREEPM_ERR_ARG, "a box appears twice in the batch");
        if (c->device != lead->device)
            return fail(c, TREEPM_ERR_ARG, "the boxes of a batch share one device");
        if (c->state < 1) return fail(c, TREEPM_ERR_STATE, "treepm_force_short_batch needs a build");
        if (c->prm.precision != TREEPM_FP32)
            return fail(c, TREEPM_ERR_ARG, "shared launches run the FP32 path only");
        if (!ax[b] || !ay[b] || !az[b]) return fail(c, TREEPM_ERR_ARG, "NULL output buffer");
        if (mem_kind != TREEPM_HOST && mem_kind != TREEPM_DEVICE)
            return fail(c, TREEPM_ERR_ARG, "mem_kind must be TREEPM_HOST or TREEPM_DEVICE");
        const double half_side = 0.5 * std::ldexp(c->prm.L, -(int)c->min_group_level);
        if (half_side + c->prm.r_cut > 0.5 * c->prm.L)
            return fail(c, TREEPM_ERR_ARG,
                        "FP32 path needs group cube half-side + r_cut <= L/2 (a group at "
                        "level %u is too large for r_cut); use TREEPM_FP64",
                        c->min_group_level);
    }
    HIPCHK(lead, hipSetDevice(lead->device));
    hipStream_t s = (hipStream_t)hip_stream;
    BatchScope scope{ctxs, n_boxes, s};
    int rc = batch_walk(ctxs, n_boxes, s);
    if (!rc) {
        for (int b = 0; b < n_boxes; ++b) ctxs[b]->state = 2;
        rc = batch_force(ctxs, n_boxes, ax, ay, az, mem_kind, s);
    }
    if (rc) {
        // the failing box named the error; the others are left built, to be walked again
        for (int b = 0; b < n_boxes; ++b) {
            ctxs[b]->state = std::min(ctxs[b]->state, 1);
            if (ctxs[b]->err.empty()) ctxs[b]->err = "another box of the batch failed";
        }
        (void)hipStreamSynchronize(s);
    }
    return rc;
}

static bool device_array(const void *p, int device);

TREEPM_API int treepm_kick_short(treepm_ctx *c, double *vx, double *vy, double *vz, double dt,
                                 void *hip_stream)
{
    if (!c) return TREEPM_ERR_ARG;
    if (c->state < 2) return fail(c, TREEPM_ERR_STATE, "treepm_kick_short needs a walk");
    c->err.clear();
    if (!vx || !vy || !vz) return fail(c, TREEPM_ERR_ARG, "NULL velocity array");
    if (!std::isfinite(dt)) return fail(c, TREEPM_ERR_ARG, "dt must be finite");
    if (c->prm.quadrupole)
        return fail(c, TREEPM_ERR_ARG, "treepm_kick_short does not take quadrupole boxes");
    HIPCHK(c, hipSetDevice(c->device));
    for (const void *p : {(const void *)vx, (const void *)vy, (const void *)vz})
        if (!device_array(p, c->device))
            return fail(c, TREEPM_ERR_ARG, "treepm_kick_short takes device arrays");
    return do_force_short(c, vx, vy, vz, 2, TREEPM_DEVICE, hip_stream, dt);
}

TREEPM_API int treepm_force_long(treepm_ctx *c, void *ax, void *ay, void *az, int out_prec,
                                 int mem_kind, int accumulate, void *hip_stream)
{
    if (!c) return TREEPM_ERR_ARG;
    if (c->state < 1) return fail(c, TREEPM_ERR_STATE, "treepm_force_long needs a build");
    c->err.clear();
    if (!ax || !ay || !az) return fail(c, TREEPM_ERR_ARG, "NULL output buffer");
    if (out_prec != TREEPM_FP32 && out_prec != TREEPM_FP64)
        return fail(c, TREEPM_ERR_ARG, "out_prec must be TREEPM_FP32 or TREEPM_FP64");
    if (mem_kind != TREEPM_HOST && mem_kind != TREEPM_DEVICE)
        return fail(c, TREEPM_ERR_ARG, "mem_kind must be TREEPM_HOST or TREEPM_DEVICE");
    if (accumulate != 0 && accumulate != 1)
        return fail(c, TREEPM_ERR_ARG, "accumulate must be 0 or 1");
    const treepm_params &P = c->prm;
    const double q = P.L / P.mesh;
    const long long N = std::llround(q);
    if (std::fabs(q - (double)N) > 1e-9 * q || N < 16 || N > 1024 || (N & (N - 1)))
        return fail(c, TREEPM_ERR_ARG,
                    "the PM mesh N_PM = L / mesh must be a power of two in [16, 1024] (%.6g)", q);
    HIPCHK(c, hipSetDevice(c->device));
    hipStream_t s = (hipStream_t)hip_stream;
    c->last = s;
    CallScope scope(c, s);
    const size_t pts = (size_t)N * N * N, H = (size_t)N / 2 + 1;
    {
        hipError_t e = reserve(c->pm_mass, pts * 8);
        if (e == hipSuccess) e = reserve(c->pm_grid, pts * 8);
        if (e == hipSuccess) e = reserve(c->pm_f, pts * 16);
        if (e == hipSuccess) e = reserve(c->pm_green, H * H * H * 4);
        if (e == hipSuccess) e = reserve(c->pm_tw, (size_t)N / 2 * 8);
        if (e == hipSuccess) e = reserve(c->pm_stage, (size_t)c->n * 16);
        const size_t cells = pm_assign_cells((int)N);
        if (e == hipSuccess)
            e = reserve(c->pm_cells, (2 * (cells + 1) + scan_tmp_elems(cells) + 64) * 4);
        if (e == hipSuccess)
            e = reserve(c->pm_slots, pm_assign_items_max((int)N, c->n) *
                                         pm_assign_slot_words() * 8);
        if (e != hipSuccess) return hip_fail(c, e, "PM meshes");
    }
    const double eta = 0.5 * P.r_cut;
    if (c->pm_n != (int)N || c->pm_L != P.L || c->pm_eta != eta) {
        launch_pm_green((int)N, P.L, eta, c->pm_green.as<float>(), c->pm_tw.as<float2>(), s);
        c->pm_n = (int)N;
        c->pm_L = P.L;
        c->pm_eta = eta;
    }
    size_t esz = out_prec == TREEPM_FP64 ? 8 : 4;
    void *dst[3] = {ax, ay, az};
    void *const host_out[3] = {ax, ay, az};
    if (mem_kind == TREEPM_HOST) {
        for (int a = 0; a < 3; ++a) {
            hipError_t e = reserve(c->out[a], (size_t)c->n * esz);
            if (e != hipSuccess) return hip_fail(c, e, "output staging");
            dst[a] = c->out[a].p;
            if (accumulate) // the sum starts from what the caller's arrays hold
                HIPCHK(c, hipMemcpyAsync(dst[a], host_out[a], (size_t)c->n * esz,
                                         hipMemcpyHostToDevice, s));
        }
    }
    const double4 *ps = c->psrc.as<double4>();
    unsigned long long *mass = c->pm_mass.as<unsigned long long>();
    float2 *grid = c->pm_grid.as<float2>();
    float *phi = c->pm_mass.as<float>(); // the masses are consumed by the first pass
    const size_t cells = pm_assign_cells((int)N);
    uint32_t *cell_start = c->pm_cells.as<uint32_t>();
    uint32_t *item_start = cell_start + (cells + 1);
    uint32_t *scan_tmp = item_start + (cells + 1);
    launch_pm_assign(ps, c->key.as<uint64_t>(), c->n, (int)N, P.L,
                     c->pm_mx.as<unsigned long long>(), cell_start, item_start, scan_tmp,
                     c->pm_slots.as<unsigned long long>(), mass, s);
    launch_pm_potential(mass, c->pm_mx.as<unsigned long long>(), c->n, (int)N, grid, phi,
                        c->pm_green.as<float>(), c->pm_tw.as<float2>(), s);
    launch_pm_force(phi, (int)N, P.L, c->pm_f.as<float4>(), s);
    launch_pm_interp(ps, c->n, (int)N, P.L, c->pm_f.as<float4>(), c->idx.as<uint32_t>(),
                     c->pm_stage.as<float4>(), cell_start, item_start, s);
    launch_pm_split(c->pm_stage.as<float4>(), c->n, dst[0], dst[1], dst[2],
                    out_prec == TREEPM_FP64, accumulate, s);
    HIPCHK(c, hipGetLastError());
    if (mem_kind == TREEPM_HOST) {
        for (int a = 0; a < 3; ++a)
            HIPCHK(c, hipMemcpyAsync(host_out[a], dst[a], (size_t)c->n * esz,
                                     hipMemcpyDeviceToHost, s));
        HIPCHK(c, hipStreamSynchronize(s));
    }
    return TREEPM_OK;
}

// True if p is device (or managed) memory of device `device`: the time-stepping kernels read
// and write their arrays directly, so a host pointer is refused before any launch.
static bool device_array(const void *p, int device)
{
    hipPointerAttribute_t a{};
    if (hipPointerGetAttributes(&a, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return (a.type == hipMemoryTypeDevice || a.isManaged) && a.device == device;
}

TREEPM_API double treepm_eps_of_z(double z, double eps_fin, double z_crit)
{
    return z >= z_crit ? (1.0 + z_crit) / (1.0 + z) * eps_fin : eps_fin;
}

namespace {

// Argument checks shared by the two time-step entry points.
int check_timestep(treepm_ctx *c, int64_t n, const double *vx, const double *vy,
                   const double *vz, const void *ax, const void *ay, const void *az,
                   int acc_prec, double eps, double zeta, double *dt)
{
    if (!dt) return fail(c, TREEPM_ERR_ARG, "dt is NULL");
    if (n < 1 || n > 0x7fffffffLL) return fail(c, TREEPM_ERR_ARG, "n must be in [1, 2^31)");
    if (!vx || !vy || !vz || !ax || !ay || !az) return fail(c, TREEPM_ERR_ARG, "NULL buffer");
    if (acc_prec != TREEPM_FP32 && acc_prec != TREEPM_FP64)
        return fail(c, TREEPM_ERR_ARG, "acc_prec must be TREEPM_FP32 or TREEPM_FP64");
    if (!std::isfinite(eps) || !(eps > 0.0) || !std::isfinite(zeta) || !(zeta > 0.0))
        return fail(c, TREEPM_ERR_ARG, "eps and zeta must be finite and > 0");
    HIPCHK(c, hipSetDevice(c->device));
    for (const void *p : {(const void *)vx, (const void *)vy, (const void *)vz, ax, ay, az})
        if (!device_array(p, c->device))
            return fail(c, TREEPM_ERR_ARG, "treepm_timestep takes device arrays");
    return TREEPM_OK;
}

// The reduction into the device word `word`, then dt = zeta * min from its bit pattern.
int run_timestep(treepm_ctx *c, int64_t n, const double *vx, const double *vy,
                 const double *vz, const void *ax, const void *ay, const void *az,
                 int acc_prec, double eps, double zeta, hipStream_t s, unsigned long long *word,
                 double *dt)
{
    launch_timestep(n, vx, vy, vz, ax, ay, az, acc_prec == TREEPM_FP64, eps, word, s);
    HIPCHK(c, hipGetLastError());
    unsigned long long bits = 0;
    int rc = fetch(c, s, {&bits, word, sizeof bits});
    if (rc) return rc;
    double m;
    std::memcpy(&m, &bits, sizeof m);
    *dt = zeta * m;
    return TREEPM_OK;
}

} // namespace

TREEPM_API int treepm_timestep(treepm_ctx *c, int64_t n, const double *vx, const double *vy,
                               const double *vz, const void *ax, const void *ay, const void *az,
                               int acc_prec, double eps, double zeta, void *hip_stream,
                               double *dt)
{
    if (!c) return TREEPM_ERR_ARG;
    c->err.clear();
    int rc = check_timestep(c, n, vx, vy, vz, ax, ay, az, acc_prec, eps, zeta, dt);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)hip_stream;
    c->last = s;
    CallScope scope(c, s);
    {
        hipError_t e = reserve(c->step_min, 8);
        if (e != hipSuccess) return hip_fail(c, e, "time step");
    }
    return run_timestep(c, n, vx, vy, vz, ax, ay, az, acc_prec, eps, zeta, s,
                        c->step_min.as<unsigned long long>(), dt);
}

TREEPM_API int treepm_timestep_noalloc(treepm_ctx *c, int64_t n, const double *vx,
                                       const double *vy, const double *vz, const void *ax,
                                       const void *ay, const void *az, int acc_prec, double eps,
                                       double zeta, void *hip_stream, double *dt)
{
    if (!c) return TREEPM_ERR_ARG;
    c->err.clear();
    int rc = check_timestep(c, n, vx, vy, vz, ax, ay, az, acc_prec, eps, zeta, dt);
    if (rc) return rc;
    unsigned long long *word = nullptr;
    {
        const hipError_t e = step_scratch(c->device, &word);
        if (e != hipSuccess) return hip_fail(c, e, "device scratch of the time step");
    }
    hipStream_t s = (hipStream_t)hip_stream;
    c->last = s;
    CallScope scope(c, s);
    return run_timestep(c, n, vx, vy, vz, ax, ay, az, acc_prec, eps, zeta, s, word, dt);
}

TREEPM_API int treepm_kick_drift(treepm_ctx *c, int64_t n, double *x, double *y, double *z,
                                 double *vx, double *vy, double *vz, const void *ax,
                                 const void *ay, const void *az, int acc_prec, double dt_kick,
                                 double dt_drift, void *hip_stream)
{
    if (!c) return TREEPM_ERR_ARG;
    c->err.clear();
    if (n < 1 || n > 0x7fffffffLL) return fail(c, TREEPM_ERR_ARG, "n must be in [1, 2^31)");
    if (!x || !y || !z || !vx || !vy || !vz || !ax || !ay || !az)
        return fail(c, TREEPM_ERR_ARG, "NULL buffer");
    if (acc_prec != TREEPM_FP32 && acc_prec != TREEPM_FP64)
        return fail(c, TREEPM_ERR_ARG, "acc_prec must be TREEPM_FP32 or TREEPM_FP64");
    if (!std::isfinite(dt_kick) || !std::isfinite(dt_drift))
        return fail(c, TREEPM_ERR_ARG, "dt_kick and dt_drift must be finite");
    HIPCHK(c, hipSetDevice(c->device));
    for (const void *p : {(const void *)x, (const void *)y, (const void *)z, (const void *)vx,
                          (const void *)vy, (const void *)vz, ax, ay, az})
        if (!device_array(p, c->device))
            return fail(c, TREEPM_ERR_ARG, "treepm_kick_drift takes device arrays");
    hipStream_t s = (hipStream_t)hip_stream;
    c->last = s;
    CallScope scope(c, s);
    launch_kick_drift(n, x, y, z, vx, vy, vz, ax, ay, az, acc_prec == TREEPM_FP64, dt_kick,
                      dt_drift, c->prm.L, s);
    HIPCHK(c, hipGetLastError());
    return TREEPM_OK;
}

TREEPM_API int treepm_get_stats(treepm_ctx *c, treepm_stats *stats)
{
    if (!c || !stats) return TREEPM_ERR_ARG;
    HIPCHK(c, hipSetDevice(c->device));
    if (c->timing) HIPCHK(c, hipStreamSynchronize(c->last));
    fill_stats(c, stats);
    if (c->state >= 2 && c->last_force_prec >= 0) {
        unsigned long long ev = 0;
        int rc = d2h(c, &ev, c->kept_sum.p, 1, c->last);
        if (rc) return rc;
        stats->evaluated = (int64_t)ev;
    }
    return TREEPM_OK;
}

TREEPM_API int treepm_export_sorted(treepm_ctx *c, uint64_t *keys, int64_t *idx)
{
    if (!c || !keys || !idx) return TREEPM_ERR_ARG;
    if (c->state < 1) return fail(c, TREEPM_ERR_STATE, "no build");
    HIPCHK(c, hipSetDevice(c->device));
    int rc;
    size_t n = (size_t)c->n;
    if ((rc = d2h(c, keys, c->key.p, n, c->last))) return rc;
    std::vector<uint32_t> i32(n);
    if ((rc = d2h(c, i32.data(), c->idx.p, n, c->last))) return rc;
    for (size_t k = 0; k < n; ++k) idx[k] = i32[k];
    return TREEPM_OK;
}

TREEPM_API int treepm_export_nodes(treepm_ctx *c, int64_t cap, uint64_t *code, int64_t *first,
                                   int64_t *count, int32_t *nchild, double *mass, double *com)
{
    if (!c || !code || !first || !count || !nchild || !mass || !com) return TREEPM_ERR_ARG;
    if (c->state < 1) return fail(c, TREEPM_ERR_STATE, "no build");
    if (cap < (int64_t)c->n_nodes) return fail(c, TREEPM_ERR_ARG, "cap < n_nodes");
    HIPCHK(c, hipSetDevice(c->device));
    int rc;
    size_t nn = c->n_nodes;
    hipStream_t s = c->last;
    std::vector<uint32_t> u(nn);
    std::vector<uint8_t> b(nn);
    std::vector<double> d(nn);
    if ((rc = d2h(c, code, c->n_code.p, nn, s))) return rc;
    if ((rc = d2h(c, u.data(), c->n_first.p, nn, s))) return rc;
    for (size_t k = 0; k < nn; ++k) first[k] = u[k];
    if ((rc = d2h(c, u.data(), c->n_count.p, nn, s))) return rc;
    for (size_t k = 0; k < nn; ++k) count[k] = u[k];
    if ((rc = d2h(c, b.data(), c->n_nch.p, nn, s))) return rc;
    for (size_t k = 0; k < nn; ++k) nchild[k] = b[k];
    if ((rc = d2h(c, mass, c->n_mass.p, nn, s))) return rc;
    std::vector<double> src(4 * nn); // (centre of mass, mass) per node
    if ((rc = d2h(c, src.data(), c->n_src.p, 4 * nn, s))) return rc;
    for (size_t k = 0; k < nn; ++k)
        for (int a = 0; a < 3; ++a) com[3 * k + a] = src[4 * k + a];
    return TREEPM_OK;
}

TREEPM_API int treepm_export_groups(treepm_ctx *c, int64_t cap, uint64_t *code, int64_t *first,
                                    int64_t *count, double *lo, double *hi, double *xg)
{
    if (!c || !code || !first || !count || !lo || !hi || !xg) return TREEPM_ERR_ARG;
    if (c->state < 1) return fail(c, TREEPM_ERR_STATE, "no build");
    if (cap < (int64_t)c->n_groups) return fail(c, TREEPM_ERR_ARG, "cap < n_groups");
    HIPCHK(c, hipSetDevice(c->device));
    int rc;
    size_t ng = c->n_groups, nn = c->n_nodes;
    hipStream_t s = c->last;
    std::vector<uint32_t> u(ng);
    std::vector<uint64_t> codes(nn);
    std::vector<double> d(ng);
    if ((rc = d2h(c, codes.data(), c->n_code.p, nn, s))) return rc;
    if ((rc = d2h(c, u.data(), c->g_node.p, ng, s))) return rc;
    for (size_t g = 0; g < ng; ++g) code[g] = codes[u[g]];
    if ((rc = d2h(c, u.data(), c->g_first.p, ng, s))) return rc;
    for (size_t g = 0; g < ng; ++g) first[g] = u[g];
    if ((rc = d2h(c, u.data(), c->g_count.p, ng, s))) return rc;
    for (size_t g = 0; g < ng; ++g) count[g] = u[g];
    Buf *srcs[3][3] = {{&c->g_lo[0], &c->g_lo[1], &c->g_lo[2]},
                       {&c->g_hi[0], &c->g_hi[1], &c->g_hi[2]},
                       {&c->g_xg[0], &c->g_xg[1], &c->g_xg[2]}};
    double *dsts[3] = {lo, hi, xg};
    for (int q = 0; q < 3; ++q)
        for (int a = 0; a < 3; ++a) {
            if ((rc = d2h(c, d.data(), srcs[q][a]->p, ng, s))) return rc;
            for (size_t g = 0; g < ng; ++g) dsts[q][3 * g + a] = d[g];
        }
    return TREEPM_OK;
}

TREEPM_API int treepm_export_lists(treepm_ctx *c, int64_t group_cap, int64_t entry_cap,
                                   int64_t *offsets, uint8_t *is_cell, uint64_t *value)
{
    if (!c || !offsets || !is_cell || !value) return TREEPM_ERR_ARG;
    if (c->state < 2) return fail(c, TREEPM_ERR_STATE, "no walk");
    if (group_cap < (int64_t)c->n_groups + 1 || entry_cap < (int64_t)c->n_entries)
        return fail(c, TREEPM_ERR_ARG, "capacity too small (%lld groups, %llu entries)",
                    (long long)c->n_groups, (unsigned long long)c->n_entries);
    HIPCHK(c, hipSetDevice(c->device));
    int rc;
    hipStream_t s = c->last;
    size_t ng = c->n_groups, nn = c->n_nodes, ne = c->n_entries, n = c->n;
    std::vector<uint64_t> off(ng + 1), codes(nn);
    std::vector<uint32_t> len(ng + 1), idx(n);
    if ((rc = d2h(c, off.data(), c->off.p, ng, s))) return rc;
    if ((rc = d2h(c, len.data(), c->glen.p, ng, s))) return rc;
    if ((rc = d2h(c, codes.data(), c->n_code.p, nn, s))) return rc;
    if ((rc = d2h(c, idx.data(), c->idx.p, n, s))) return rc;
    // lists may sit anywhere in the entries buffer: copy the used span, write them back to back
    size_t span = 0;
    for (size_t g = 0; g < ng; ++g) span = std::max<size_t>(span, off[g] + len[g]);
    std::vector<uint32_t> ent(span);
    if (span && (rc = d2h(c, ent.data(), c->entries.p, span, s))) return rc;
    size_t q = 0;
    for (size_t g = 0; g < ng; ++g) {
        offsets[g] = (int64_t)q;
        for (uint32_t j = 0; j < len[g]; ++j, ++q) {
            const uint32_t e = ent[off[g] + j];
            if (e & kCellTag) {
                is_cell[q] = 1;
                value[q] = codes[e & ~kCellTag];
            } else {
                is_cell[q] = 0;
                value[q] = idx[e];
            }
        }
    }
    offsets[ng] = (int64_t)q;
    if (q != ne) return fail(c, TREEPM_ERR_STATE, "list lengths do not add up");
    return TREEPM_OK;
}

TREEPM_API int treepm_autotune(treepm_ctx *c, int64_t n, const double *x, const double *y,
                               const double *z, const double *m, int mem_kind, void *hip_stream,
                               const int32_t *candidates, int32_t n_candidates, int32_t *best,
                               double *best_ms)
{
    if (!c || !candidates || n_candidates < 1 || n_candidates > 64) return TREEPM_ERR_ARG;
    for (int i = 0; i < n_candidates; ++i)
        if (candidates[i] < 1) return fail(c, TREEPM_ERR_ARG, "n_crit candidates must be >= 1");
    int rc;
    HIPCHK(c, hipSetDevice(c->device));
    hipStream_t s = (hipStream_t)hip_stream;
    // device outputs for the trial forces (their values are discarded)
    Buf tmp[3];
    {
        CallScope scope(c, s);
        for (Buf &b : tmp) {
            hipError_t e = reserve(b, (size_t)n * 4);
            if (e != hipSuccess) {
                for (Buf &q : tmp) release(q);
                return hip_fail(c, e, "autotune outputs");
            }
        }
    }
    hipEvent_t e0, e1;
    HIPCHK(c, hipEventCreate(&e0));
    HIPCHK(c, hipEventCreate(&e1));
    const treepm_params base = c->prm;
    int32_t win = candidates[0];
    double win_ms = 1e300;
    rc = TREEPM_OK;
    for (int i = 0; i < n_candidates && !rc; ++i) {
        c->prm.n_crit = candidates[i];
        float best_t = 1e30f;
        for (int rep = 0; rep < 2 && !rc; ++rep) {
            (void)hipEventRecord(e0, s);
            rc = treepm_build(c, n, x, y, z, m, mem_kind, s);
            if (!rc) rc = treepm_walk(c, s, nullptr);
            if (!rc)
                rc = treepm_force_short(c, tmp[0].p, tmp[1].p, tmp[2].p, TREEPM_FP32,
                                        TREEPM_DEVICE, s);
            (void)hipEventRecord(e1, s);
            if (!rc && hipEventSynchronize(e1) == hipSuccess) {
                float t = 0.f;
                if (hipEventElapsedTime(&t, e0, e1) == hipSuccess && rep > 0) best_t = t;
            }
        }
        if (!rc && best_t < win_ms) {
            win_ms = best_t;
            win = candidates[i];
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    {
        CallScope scope(c, s);
        for (Buf &b : tmp) release(b);
    }
    c->prm = base;
    c->prm.n_crit = win;
    if (rc) return rc;
    // leave the context built and walked with the winner
    rc = treepm_build(c, n, x, y, z, m, mem_kind, s);
    if (!rc) rc = treepm_walk(c, s, nullptr);
    if (rc) return rc;
    if (best) *best = win;
    if (best_ms) *best_ms = win_ms;
    return TREEPM_OK;
}

TREEPM_API int treepm_pairwise_f32(const treepm_params *params, int device, int64_t n_i,
                                   const double *xi, int64_t n_j, const double *xj,
                                   const double *mj, const double *xg, double *out)
{
    int rc = check_params(nullptr, params);
    if (rc) return rc;
    if (n_i < 1 || n_j < 1 || n_i * n_j > (int64_t)1 << 28 || !xi || !xj || !mj || !xg || !out)
        return TREEPM_ERR_ARG;
    std::vector<float4> coef;
    uint32_t tbase = 0;
    float tc = 0.f;
    if (!build_force_table(params->eps / params->r_cut, coef, tbase, tc))
        return TREEPM_ERR_ARG;
    if (hipSetDevice(device) != hipSuccess) return TREEPM_ERR_DEVICE;
    size_t bt = coef.size() * sizeof(float4), bi = (size_t)n_i * 3 * 8,
           bj = (size_t)n_j * 3 * 8, bm = (size_t)n_j * 8, bo = (size_t)n_i * n_j * 3 * 8;
    char *d = nullptr;
    if (hipMalloc(&d, bt + bi + bj + bm + bo) != hipSuccess) return TREEPM_ERR_OOM;
    float4 *dtab = (float4 *)d;
    double *dxi = (double *)(d + bt), *dxj = (double *)(d + bt + bi),
           *dmj = (double *)(d + bt + bi + bj), *dout = (double *)(d + bt + bi + bj + bm);
    hipError_t e = hipMemcpy(dtab, coef.data(), bt, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(dxi, xi, bi, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(dxj, xj, bj, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(dmj, mj, bm, hipMemcpyHostToDevice);
    if (e == hipSuccess) {
        const ForceTable ft{dtab, (uint32_t)coef.size(), tbase, tc};
        launch_pairwise_f32(n_i, dxi, n_j, dxj, dmj, xg, 0.5 * params->r_cut, ft, dout,
                            nullptr);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpy(out, dout, bo, hipMemcpyDeviceToHost);
    (void)hipFree(d);
    return e == hipSuccess ? TREEPM_OK : TREEPM_ERR_DEVICE;
}

TREEPM_API const char *treepm_last_error(const treepm_ctx *c)
{
    return c ? c->err.c_str() : "NULL context";
}
