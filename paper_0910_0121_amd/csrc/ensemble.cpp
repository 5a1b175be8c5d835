// Ensemble server: force evaluations for many independent periodic boxes, admitted by an
// HBM budget, run concurrently on one GPU.
//
// submit() copies a request's inputs and queues it.  max_inflight worker threads each own a
// HIP stream and pinned staging buffers; a worker takes the first queued request that can
// run now -- its box is not busy with another request, and the box is already resident or
// its estimated footprint fits in the budget after evicting idle boxes, least recently used
// first -- and runs build, walk and FP32 force for it on its stream.  A box's context (its
// device buffers: particles, tree, lists) stays resident between requests until evicted.
// Requests from different workers overlap on the device.  poll() is non-blocking.
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
        if (hipHostMalloc(&p, c) != hipSuccess) return nullptr;
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

struct Request {
    uint64_t ticket = 0, box_id = 0;
    treepm_params prm{};
    int64_t n = 0;
    double *in = nullptr; // pinned: x, y, z, m blocks
    size_t in_cap = 0;
    float *out = nullptr; // pinned: ax, ay, az blocks
    size_t out_cap = 0;
    int state = 0; // 0 queued, 1 running, 2 done
    int rc = 0;
    treepm_stats stats{};
    double t_submit = 0, t_start = 0, t_done = 0;
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

int run_request(treepm_ens *e, Worker &w, Request &r, Box &b)
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
    const double *x = r.in, *y = x + r.n, *z = y + r.n, *m = z + r.n;
    rc = treepm_build(b.ctx, r.n, x, y, z, m, TREEPM_HOST, w.stream);
    // no copy from the pinned inputs may still be in flight when the block is reused
    hipError_t se = hipStreamSynchronize(w.stream);
    if (!rc && se != hipSuccess) rc = TREEPM_ERR_DEVICE;
    e->pool.put(r.in, r.in_cap);
    r.in = nullptr;
    if (rc) return rc;
    rc = treepm_walk(b.ctx, w.stream, nullptr);
    if (rc) return rc;
    r.out = (float *)e->pool.get((size_t)r.n * 3 * sizeof(float), &r.out_cap);
    if (!r.out) return TREEPM_ERR_OOM;
    float *ax = r.out, *ay = ax + r.n, *az = ay + r.n;
    rc = treepm_force_short(b.ctx, ax, ay, az, TREEPM_FP32, TREEPM_HOST, w.stream);
    if (rc) return rc;
    rc = treepm_get_stats(b.ctx, &r.stats);
    if (rc) return rc;
    return TREEPM_OK;
}

void worker_main(treepm_ens *e, int wi)
{
    hipSetDevice(e->device);
    Worker &w = e->workers[wi];
    hipStreamCreateWithFlags(&w.stream, hipStreamNonBlocking);
    for (;;) {
        std::shared_ptr<Request> r;
        std::vector<treepm_ctx *> gone;
        bool quit = false;
        {
            std::unique_lock<std::mutex> lk(e->mu);
            // also wake for contexts evicted on the way, to destroy them promptly
            e->cv.wait(lk, [&] {
                if (e->stop) return true;
                r = pick(e, gone);
                return r != nullptr || !gone.empty();
            });
            if (r) {
                r->state = 1;
                r->t_start = now_s();
                ++e->inflight;
            } else {
                quit = e->stop;
            }
        }
        for (treepm_ctx *g : gone) treepm_destroy(g); // evicted: outside the lock
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
        int rc = run_request(e, w, *r, local);
        {
            std::lock_guard<std::mutex> lk(e->mu);
            Box &b = e->boxes[r->box_id];
            b.ctx = local.ctx;
            b.prm = local.prm;
            if (b.ctx) {
                size_t actual = treepm_internal_ctx_bytes(b.ctx);
                if (actual > b.bytes) {
                    e->resident += actual - b.bytes;
                    b.bytes = actual;
                }
            }
            if (rc) { // a failed box is dropped so it cannot poison later requests
                if (b.ctx) treepm_destroy(b.ctx);
                e->resident -= std::min(e->resident, b.bytes);
                e->boxes.erase(r->box_id);
            } else {
                b.busy = false;
                b.last_use = ++e->clock;
            }
            r->rc = rc;
            r->t_done = now_s();
            r->state = 2;
            if (r->in) e->pool.put(r->in, r->in_cap);
            r->in = nullptr;
            if (rc && r->out) {
                e->pool.put(r->out, r->out_cap);
                r->out = nullptr;
            }
            --e->inflight;
        }
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
        if (kv.second->in) e->pool.put(kv.second->in, kv.second->in_cap);
        if (kv.second->out) e->pool.put(kv.second->out, kv.second->out_cap);
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
    r->in = (double *)e->pool.get((size_t)n * 4 * sizeof(double), &r->in_cap);
    if (!r->in) return TREEPM_ERR_OOM;
    double *dst[4] = {r->in, r->in + n, r->in + 2 * n, r->in + 3 * n};
    const double *src[4] = {x, y, z, m};
    copy_parallel(dst, src, 4, n);
    {
        std::lock_guard<std::mutex> lk(e->mu);
        int rc = TREEPM_OK;
        if (e->stop)
            rc = TREEPM_ERR_STATE;
        else if (e->queue.size() >= e->queue_cap)
            rc = TREEPM_ERR_QUEUE_FULL;
        if (rc) { // the pinned block goes back to the pool
            e->pool.put(r->in, r->in_cap);
            r->in = nullptr;
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
        const float *src[3] = {r->out, r->out + r->n, r->out + 2 * r->n};
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
    e->pool.put(r->out, r->out_cap);
    r->out = nullptr;
    if (stats) {
        *stats = r->stats;
        stats->latency_ms = (r->t_done - r->t_submit) * 1e3;
        stats->queue_ms = (r->t_start - r->t_submit) * 1e3;
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
