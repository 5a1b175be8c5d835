// Ensemble server: force evaluations for many independent periodic boxes, admitted by an
// HBM budget, run concurrently on one GPU with shared launches.
//
// submit() copies a request's inputs and queues it.  max_inflight worker threads each own a
// HIP stream.  A worker takes the first queued request that can run now -- its box is not
// busy with another request, and the box is already resident or its estimated footprint
// fits in the budget after evicting idle boxes, least recently used first -- and builds the
// box's tree on its stream, then runs its walk and FP32 force there.  With shared launches
// switched on (treepm_ens_set_batching) a built box instead waits in a ready list, and
// whenever no batch is running the next free worker takes every ready box (up to kMaxBatch)
// and runs their walks and forces together (treepm_force_short_batch: one traversal launch
// and one launch per size class for all of them) while the other workers build the next
// boxes.  A box's context (its device buffers: particles, tree, lists) stays resident between
// requests until evicted.  poll() is non-blocking.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <future>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "common.hpp"
#include "treepm.h"

#define TREEPM_API extern "C" __attribute__((visibility("default")))

// Device bytes a context currently holds, and the parameter checks of treepm_create, without
// a device (treepm.cpp).
size_t treepm_internal_ctx_bytes(const treepm_ctx *c);
int treepm_internal_check_params(const treepm_params *p);

namespace {

double now_s()
{
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

// Conservative device footprint of one box of n particles before its first build: particle
// arrays and sort buffers (~100 B), tree (~60 B), groups, and interaction lists (~150 B).
size_t estimate_bytes(int64_t n) { return (size_t)n * 320 + ((size_t)64 << 20); }

// Pinned host blocks, reused across requests (sizes rounded up to a power of two), so a
// request neither page-faults fresh memory nor needs a second staging copy.  A request takes
// the smallest free block that holds it and is at most four times its size: pinning fresh
// memory is slow for a large block (hundreds of ms) and holds up other HIP calls meanwhile,
// while a small one is cheap to pin and should not take a block a large request needs.
class PinnedPool {
  public:
    ~PinnedPool()
    {
        for (auto &kv : free_) hipHostFree(kv.second);
    }
    void *get(size_t bytes, size_t *cap)
    {
        size_t c = (size_t)1 << 20;
        while (c < bytes) c <<= 1;
        {
            std::lock_guard<std::mutex> lk(mu_);
            auto it = free_.lower_bound(c);
            if (it != free_.end() && it->first <= 4 * c) {
                c = it->first;
                void *p = it->second;
                free_.erase(it);
                *cap = c;
                return p;
            }
        }
        void *p = nullptr;
        if (hipHostMalloc(&p, c) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        *cap = c;
        return p;
    }
    void put(void *p, size_t cap)
    {
        if (!p) return;
        std::lock_guard<std::mutex> lk(mu_);
        free_.emplace(cap, p);
    }

  private:
    std::mutex mu_;
    std::multimap<size_t, void *> free_;
};

// A pinned host block from the pool (p is null if pinning failed).
struct HostBlock {
    void *p = nullptr;
    size_t cap = 0;
};

HostBlock take_block(PinnedPool &pool, size_t bytes)
{
    HostBlock b;
    b.p = pool.get(bytes, &b.cap);
    return b;
}

void give_block(PinnedPool &pool, HostBlock &b)
{
    if (b.p) pool.put(b.p, b.cap);
    b = HostBlock{};
}

struct Request {
    uint64_t ticket = 0, box_id = 0;
    treepm_params prm{};
    int64_t n = 0;
    HostBlock in;  // x, y, z, m blocks of n doubles
    HostBlock out; // ax, ay, az blocks of n floats
    int state = 0; // 0 queued, 1 running, 2 done
    int rc = 0;
    int batch = 1; // boxes that shared the walk and force launches
    treepm_ctx *ctx = nullptr; // the box's context while the request runs
    treepm_stats stats{};
    double t_submit = 0, t_start = 0, t_built = 0, t_batch = 0, t_done = 0;
};

// Copy k arrays of n doubles/floats.  Large requests are cut into pieces of at least 4 MiB
// spread over up to kCopyThreads threads (one thread's memcpy reaches only a fraction of the
// host's memory bandwidth).
constexpr int kCopyThreads = 8;

template <typename T>
void copy_parallel(T *const *dst, const T *const *src, int k, int64_t n)
{
    const size_t bytes = (size_t)n * sizeof(T), piece_min = (size_t)4 << 20;
    const size_t total = bytes * (size_t)k;
    if (total < 2 * piece_min) {
        for (int a = 0; a < k; ++a) memcpy(dst[a], src[a], bytes);
        return;
    }
    size_t pieces = total / piece_min;
    if (pieces > (size_t)kCopyThreads) pieces = kCopyThreads;
    const size_t share = (total + pieces - 1) / pieces;
    // piece p copies bytes [p share, (p + 1) share) of the k arrays laid end to end
    auto run = [=](size_t p) {
        size_t lo = p * share, hi = std::min(total, lo + share);
        while (lo < hi) {
            const size_t a = lo / bytes, off = lo % bytes, len = std::min(hi - lo, bytes - off);
            memcpy((char *)dst[a] + off, (const char *)src[a] + off, len);
            lo += len;
        }
    };
    std::vector<std::future<void>> fs;
    for (size_t p = 1; p < pieces; ++p) fs.push_back(std::async(std::launch::async, run, p));
    run(0);
    for (auto &f : fs) f.get();
}

struct Box {
    treepm_ctx *ctx = nullptr;
    size_t bytes = 0;
    bool busy = false;
    uint64_t last_use = 0;
    treepm_params prm{};
};

struct Worker {
    hipStream_t stream = nullptr;
};

} // namespace

struct treepm_ens {
    int device = 0;
    size_t budget = 0;
    int max_inflight = 1;
    size_t queue_cap = 4096;
    std::mutex mu;
    std::condition_variable cv;
    std::deque<std::shared_ptr<Request>> queue;
    std::unordered_map<uint64_t, std::shared_ptr<Request>> tickets;
    std::unordered_map<uint64_t, Box> boxes;
    // built boxes waiting for their walk and force, and whether a batch is running
    std::vector<std::shared_ptr<Request>> ready;
    bool leading = false;
    bool batching = false; // shared launches (treepm_ens_set_batching)
    size_t resident = 0;
    uint64_t clock = 0, next_ticket = 1;
    int inflight = 0;
    bool stop = false;
    std::vector<std::thread> threads;
    std::vector<Worker> workers;
    PinnedPool pool;
};

namespace {

size_t box_need(const treepm_ens *e, const Request &r)
{
    auto it = e->boxes.find(r.box_id);
    size_t est = estimate_bytes(r.n);
    if (it == e->boxes.end()) return est;
    return it->second.bytes >= est ? 0 : est - it->second.bytes;
}

// With e->mu held: evict idle boxes (least recently used first) until `need` more bytes fit;
// their contexts go to `gone`, for the caller to destroy after releasing the lock (destroying
// waits for the context's last work).  Returns false if they cannot be made to fit now.
bool make_room(treepm_ens *e, size_t need, uint64_t keep_box, std::vector<treepm_ctx *> &gone)
{
    while (e->resident + need > e->budget) {
        uint64_t victim = 0;
        uint64_t oldest = UINT64_MAX;
        bool found = false;
        for (auto &kv : e->boxes)
            if (!kv.second.busy && kv.first != keep_box && kv.second.last_use < oldest) {
                oldest = kv.second.last_use;
                victim = kv.first;
                found = true;
            }
        if (!found) return false;
        Box &b = e->boxes[victim];
        if (b.ctx) gone.push_back(b.ctx);
        e->resident -= std::min(e->resident, b.bytes);
        e->boxes.erase(victim);
    }
    return true;
}

// With e->mu held: the first queued request that can start now, or nullptr; evicted contexts
// are added to `gone`.
std::shared_ptr<Request> pick(treepm_ens *e, std::vector<treepm_ctx *> &gone)
{
    for (auto it = e->queue.begin(); it != e->queue.end(); ++it) {
        Request &r = **it;
        auto bi = e->boxes.find(r.box_id);
        if (bi != e->boxes.end() && bi->second.busy) continue;
        size_t need = box_need(e, r);
        if (!make_room(e, need, r.box_id, gone)) continue;
        Box &b = e->boxes[r.box_id];
        b.busy = true;
        b.last_use = ++e->clock;
        e->resident += need;
        b.bytes += need;
        std::shared_ptr<Request> sel = *it;
        e->queue.erase(it);
        return sel;
    }
    return nullptr;
}

// The box's context (created, or given the request's parameters) and its tree, built from
// the request's inputs on the worker's stream.
int build_request(treepm_ens *e, Worker &w, Request &r, Box &b)
{
    int rc;
    if (!b.ctx) {
        rc = treepm_create(&r.prm, e->device, &b.ctx);
        if (rc) return rc;
        b.prm = r.prm;
    } else if (memcmp(&b.prm, &r.prm, sizeof r.prm) != 0) {
        rc = treepm_set_params(b.ctx, &r.prm);
        if (rc) return rc;
        b.prm = r.prm;
    }
    const double *x = static_cast<const double *>(r.in.p), *y = x + r.n, *z = y + r.n,
                 *m = z + r.n;
    // returns once the inputs have been copied and the tree is built
    rc = treepm_build(b.ctx, r.n, x, y, z, m, TREEPM_HOST, w.stream);
    give_block(e->pool, r.in);
    return rc;
}

// Walk and force of the ready boxes `batch` with shared launches; if the batch call fails,
// each box runs alone so that the failure stays with the box that caused it.
void run_batch(treepm_ens *e, Worker &w, std::vector<std::shared_ptr<Request>> &batch)
{
    const int nb = (int)batch.size();
    std::vector<treepm_ctx *> ctxs;
    std::vector<float *> ax, ay, az;
    std::vector<std::shared_ptr<Request>> run;
    for (auto &r : batch) {
        r->t_batch = now_s();
        r->out = take_block(e->pool, (size_t)r->n * 3 * sizeof(float));
        if (!r->out.p) {
            r->rc = TREEPM_ERR_OOM;
            continue;
        }
        float *o = static_cast<float *>(r->out.p);
        ctxs.push_back(r->ctx);
        ax.push_back(o);
        ay.push_back(o + r->n);
        az.push_back(o + 2 * r->n);
        run.push_back(r);
    }
    if (run.empty()) return;
    int rc = treepm_force_short_batch(ctxs.data(), (int)run.size(), ax.data(), ay.data(),
                                      az.data(), TREEPM_HOST, w.stream);
    for (size_t k = 0; k < run.size(); ++k) {
        Request &r = *run[k];
        int rk = rc;
        r.batch = rc ? 1 : (int)run.size();
        if (rc) {
            rk = treepm_walk(r.ctx, w.stream, nullptr);
            if (!rk)
                rk = treepm_force_short(r.ctx, ax[k], ay[k], az[k], TREEPM_FP32, TREEPM_HOST,
                                        w.stream);
        }
        if (!rk) rk = treepm_get_stats(r.ctx, &r.stats);
        r.rc = rk;
    }
    (void)nb;
}

// Walk and force of one built box alone, on the worker's stream.
void run_alone(treepm_ens *e, Worker &w, Request &r)
{
    r.t_batch = now_s();
    r.batch = 1;
    r.out = take_block(e->pool, (size_t)r.n * 3 * sizeof(float));
    if (!r.out.p) {
        r.rc = TREEPM_ERR_OOM;
        return;
    }
    float *o = static_cast<float *>(r.out.p);
    int rc = treepm_walk(r.ctx, w.stream, nullptr);
    if (!rc) rc = treepm_force_short(r.ctx, o, o + r.n, o + 2 * r.n, TREEPM_FP32, TREEPM_HOST,
                                     w.stream);
    if (!rc) rc = treepm_get_stats(r.ctx, &r.stats);
    r.rc = rc;
}

// With e->mu held: request r is over (rc set); its box becomes idle, or is dropped (its
// context to `gone`) if the request failed, so that it cannot poison later requests.
void finish(treepm_ens *e, Request &r, std::vector<treepm_ctx *> &gone)
{
    Box &b = e->boxes[r.box_id];
    if (b.ctx) {
        size_t actual = treepm_internal_ctx_bytes(b.ctx);
        if (actual > b.bytes) {
            e->resident += actual - b.bytes;
            b.bytes = actual;
        }
    }
    if (r.rc) {
        if (b.ctx) gone.push_back(b.ctx);
        e->resident -= std::min(e->resident, b.bytes);
        e->boxes.erase(r.box_id);
        give_block(e->pool, r.out);
    } else {
        b.busy = false;
        b.last_use = ++e->clock;
    }
    give_block(e->pool, r.in);
    r.ctx = nullptr;
    r.t_done = now_s();
    r.state = 2;
    --e->inflight;
}

void worker_main(treepm_ens *e, int wi)
{
    hipSetDevice(e->device);
    Worker &w = e->workers[wi];
    hipStreamCreateWithFlags(&w.stream, hipStreamNonBlocking);
    for (;;) {
        std::shared_ptr<Request> r;
        std::vector<std::shared_ptr<Request>> batch;
        std::vector<treepm_ctx *> gone;
        bool quit = false;
        {
            std::unique_lock<std::mutex> lk(e->mu);
            // lead a batch when built boxes wait and none runs; else build the next request;
            // also wake for contexts evicted on the way, to destroy them promptly
            e->cv.wait(lk, [&] {
                if (e->stop) return true;
                if (!e->leading && !e->ready.empty()) {
                    const size_t k = std::min<size_t>(e->ready.size(), tpm::kMaxBatch);
                    batch.assign(e->ready.begin(), e->ready.begin() + k);
                    e->ready.erase(e->ready.begin(), e->ready.begin() + k);
                    e->leading = true;
                    return true;
                }
                r = pick(e, gone);
                return r != nullptr || !gone.empty();
            });
            if (r) {
                r->state = 1;
                r->t_start = now_s();
                ++e->inflight;
            } else if (batch.empty()) {
                quit = e->stop;
            }
        }
        for (treepm_ctx *g : gone) treepm_destroy(g); // evicted: outside the lock
        gone.clear();
        if (!batch.empty()) {
            run_batch(e, w, batch);
            {
                std::lock_guard<std::mutex> lk(e->mu);
                for (auto &q : batch) finish(e, *q, gone);
                e->leading = false;
            }
            for (treepm_ctx *g : gone) treepm_destroy(g);
            e->cv.notify_all();
            continue;
        }
        if (!r) {
            if (quit) break;
            continue;
        }
        Box local;
        {
            // ctx pointer and params; nobody else touches the entry while it is busy
            std::lock_guard<std::mutex> lk(e->mu);
            local = e->boxes[r->box_id];
        }
        int rc = build_request(e, w, *r, local);
        bool alone = false;
        {
            std::lock_guard<std::mutex> lk(e->mu);
            Box &b = e->boxes[r->box_id];
            b.ctx = local.ctx;
            b.prm = local.prm;
            r->t_built = now_s();
            r->rc = rc;
            r->ctx = b.ctx;
            if (rc) {
                r->t_batch = r->t_built;
                finish(e, *r, gone);
            } else if (e->batching) {
                e->ready.push_back(r);
            } else {
                alone = true;
            }
        }
        if (alone) {
            run_alone(e, w, *r);
            std::lock_guard<std::mutex> lk(e->mu);
            finish(e, *r, gone);
        }
        for (treepm_ctx *g : gone) treepm_destroy(g);
        e->cv.notify_all();
    }
    // the stream outlives the thread: resident boxes still name it as their last stream
}

} // namespace

TREEPM_API int treepm_ens_create(int device, size_t hbm_budget, int max_inflight,
                                 treepm_ens **out)
{
    if (!out) return TREEPM_ERR_ARG;
    *out = nullptr;
    if (max_inflight < 1 || max_inflight > 16 || hbm_budget == 0) return TREEPM_ERR_ARG;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
        return TREEPM_ERR_DEVICE;
    treepm_ens *e = new (std::nothrow) treepm_ens();
    if (!e) return TREEPM_ERR_OOM;
    e->device = device;
    e->budget = hbm_budget;
    e->max_inflight = max_inflight;
    e->workers.resize(max_inflight);
    for (int i = 0; i < max_inflight; ++i) e->threads.emplace_back(worker_main, e, i);
    *out = e;
    return TREEPM_OK;
}

TREEPM_API int treepm_ens_set_batching(treepm_ens *e, int enable)
{
    if (!e || (enable != 0 && enable != 1)) return TREEPM_ERR_ARG;
    {
        std::lock_guard<std::mutex> lk(e->mu);
        e->batching = enable != 0;
    }
    e->cv.notify_all();
    return TREEPM_OK;
}

TREEPM_API int treepm_ens_destroy(treepm_ens *e)
{
    if (!e) return TREEPM_OK;
    {
        std::lock_guard<std::mutex> lk(e->mu);
        e->stop = true;
        e->queue.clear();
    }
    e->cv.notify_all();
    for (auto &t : e->threads) t.join();
    for (auto &kv : e->boxes)
        if (kv.second.ctx) treepm_destroy(kv.second.ctx);
    for (auto &w : e->workers)
        if (w.stream) (void)hipStreamDestroy(w.stream);
    for (auto &kv : e->tickets) {
        give_block(e->pool, kv.second->in);
        give_block(e->pool, kv.second->out);
    }
    e->tickets.clear();
    delete e;
    return TREEPM_OK;
}

TREEPM_API int treepm_ensemble_submit(treepm_ens *e, uint64_t box_id, const treepm_params *p,
                                      int64_t n, const double *x, const double *y,
                                      const double *z, const double *m, uint64_t *ticket)
{
    const double t_submit = now_s(); // latency counts from here
    if (!e || !p || !ticket || !x || !y || !z || !m) return TREEPM_ERR_ARG;
    if (n < 1 || n > 0x7fffffffLL) return TREEPM_ERR_ARG;
    if (p->precision != TREEPM_FP32) return TREEPM_ERR_ARG;
    {
        const int rc = treepm_internal_check_params(p);
        if (rc) return rc;
    }
    if (estimate_bytes(n) > e->budget) return TREEPM_ERR_OOM;
    auto r = std::make_shared<Request>();
    r->t_submit = t_submit;
    r->box_id = box_id;
    r->prm = *p;
    r->n = n;
    r->in = take_block(e->pool, (size_t)n * 4 * sizeof(double));
    if (!r->in.p) return TREEPM_ERR_OOM;
    double *in = static_cast<double *>(r->in.p);
    double *dst[4] = {in, in + n, in + 2 * n, in + 3 * n};
    const double *src[4] = {x, y, z, m};
    copy_parallel(dst, src, 4, n);
    {
        std::lock_guard<std::mutex> lk(e->mu);
        int rc = TREEPM_OK;
        if (e->stop)
            rc = TREEPM_ERR_STATE;
        else if (e->queue.size() >= e->queue_cap)
            rc = TREEPM_ERR_QUEUE_FULL;
        if (rc) {
            give_block(e->pool, r->in);
            return rc;
        }
        r->ticket = e->next_ticket++;
        e->queue.push_back(r);
        e->tickets[r->ticket] = r;
        *ticket = r->ticket;
    }
    e->cv.notify_all();
    return TREEPM_OK;
}

TREEPM_API int treepm_ensemble_poll(treepm_ens *e, uint64_t ticket, float *ax, float *ay,
                                    float *az, treepm_stats *stats)
{
    if (!e) return TREEPM_ERR_ARG;
    std::shared_ptr<Request> r;
    {
        std::lock_guard<std::mutex> lk(e->mu);
        auto it = e->tickets.find(ticket);
        if (it == e->tickets.end()) return TREEPM_ERR_ARG;
        if (it->second->state != 2) return TREEPM_PENDING;
        r = it->second;
        e->tickets.erase(it);
    }
    if (r->rc) return r->rc;
    {
        float *dst[3] = {ax, ay, az};
        const float *o = static_cast<const float *>(r->out.p);
        const float *src[3] = {o, o + r->n, o + 2 * r->n};
        int k = 0;
        float *d2[3];
        const float *s2[3];
        for (int a = 0; a < 3; ++a)
            if (dst[a]) {
                d2[k] = dst[a];
                s2[k] = src[a];
                ++k;
            }
        if (k) copy_parallel(d2, s2, k, r->n);
    }
    give_block(e->pool, r->out);
    if (stats) {
        *stats = r->stats;
        stats->latency_ms = (r->t_done - r->t_submit) * 1e3;
        stats->queue_ms = (r->t_start - r->t_submit) * 1e3;
        stats->stage_ms[0] = (r->t_built - r->t_start) * 1e3;
        stats->stage_ms[1] = (r->t_batch - r->t_built) * 1e3;
        stats->stage_ms[2] = (r->t_done - r->t_batch) * 1e3;
        stats->batch_boxes = r->batch;
    }
    return TREEPM_OK;
}

TREEPM_API int treepm_ens_info(treepm_ens *e, int64_t *queued, int64_t *inflight,
                               int64_t *resident_bytes, int64_t *resident_boxes)
{
    if (!e) return TREEPM_ERR_ARG;
    std::lock_guard<std::mutex> lk(e->mu);
    if (queued) *queued = (int64_t)e->queue.size();
    if (inflight) *inflight = e->inflight;
    if (resident_bytes) *resident_bytes = (int64_t)e->resident;
    if (resident_boxes) *resident_boxes = (int64_t)e->boxes.size();
    return TREEPM_OK;
}
