// Serving loop: continuous batching of fgemm requests.
//
// Requests (device-resident, caller-owned A, B, C) are queued by
// ff_server_submit.  A worker thread
//   * retires in-flight batches whose completion event has fired (their
//     requests become done, their memory is returned);
//   * admits queued requests in arrival order while their HBM footprint
//     fits the budget -- a request that does not fit yet waits, later
//     smaller ones may pass it -- and launches them as one batched
//     persistent launch on a free stream, so requests arriving while others
//     run are merged into the next launch and overlap on the device;
//   * records latency (submit to observed completion) per request.
// The footprint of a request is the HBM it touches while in flight: its
// operands and C (4(mk + kn + mn) bytes) plus its share of the batch
// workspace (digit planes or packed doubles, tables), which comes from a
// device arena of the budget's size owned by the server.
// Ordering: submit records an event on the submitting thread's stream (the
// server's opts.stream, else ff_set_stream's), and the batch that carries
// the request waits for it, so a request may be submitted right after the
// kernels that write its A, B or C are enqueued.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "ff_batch.h"

namespace ff {

namespace {

double now_s()
{
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

int64_t align256(int64_t x) { return (x + 255) & ~int64_t(255); }

// First-fit allocator over [0, size) with coalescing of free ranges.
class Arena {
  public:
    void reset(int64_t size)
    {
        free_.clear();
        if (size > 0) free_[0] = size;
        size_ = size;
    }
    bool alloc(int64_t bytes, int64_t *off)
    {
        bytes = align256(std::max<int64_t>(bytes, 256));
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const int64_t rest = it->second - bytes, at = it->first + bytes;
                free_.erase(it);
                if (rest > 0) free_[at] = rest;
                used_[*off] = bytes;
                return true;
            }
        }
        return false;
    }
    void release(int64_t off)
    {
        auto u = used_.find(off);
        if (u == used_.end()) return;
        int64_t start = off, len = u->second;
        used_.erase(u);
        auto nx = free_.lower_bound(start);
        if (nx != free_.end() && nx->first == start + len) {
            len += nx->second;
            nx = free_.erase(nx);
        }
        if (nx != free_.begin()) {
            auto pv = std::prev(nx);
            if (pv->first + pv->second == start) {
                start = pv->first;
                len += pv->second;
                free_.erase(pv);
            }
        }
        free_[start] = len;
    }

  private:
    int64_t size_ = 0;
    std::map<int64_t, int64_t> free_, used_;
};

struct Request {
    IJob job;
    int64_t footprint = 0;
    hipEvent_t ready = nullptr; // recorded on the submitting stream
    double t_submit = 0, t_done = 0;
    int state = 0; // 0 queued, 1 running, 2 done, 3 failed
    int status = FF_OK;
};

struct Inflight {
    int slot = -1;
    BatchPrep prep;
    int64_t arena_off = -1;
    std::vector<uint64_t> ids;
    int64_t footprint = 0;
};

struct Slot {
    hipStream_t st = nullptr;
    hipEvent_t done = nullptr;
    bool busy = false;
};

} // namespace

struct Server {
    int device = 0;
    ff_opts opts;
    int64_t budget = 0;
    char *arena_mem = nullptr;
    Arena arena;
    int64_t in_use = 0;
    std::vector<Slot> slots;
    std::map<int, Inflight> inflight; // by slot
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<uint64_t> queue;
    std::map<uint64_t, Request> reqs;
    uint64_t next_id = 1;
    bool stop = false;
    std::thread worker;
    // statistics
    std::vector<double> lat_ms;
    double ops = 0, t_first = -1, t_last = 0;
    int64_t running_reqs = 0, max_running = 0, completed = 0, failed = 0, submitted = 0;
    int64_t batches = 0, max_batch_seen = 0;
    int last_tile = -1;
    int max_batch = 256;
    // events for the submit-to-launch ordering, reused
    std::vector<hipEvent_t> event_pool;

    void run();
    bool retire_locked();
    bool admit_locked();
    void finish_locked(Request &r, int status, double t);
    hipEvent_t take_event_locked();
    void release_resources();
};

void Server::finish_locked(Request &r, int status, double t)
{
    r.state = status == FF_OK ? 2 : 3;
    r.status = status;
    r.t_done = t;
    if (status != FF_OK) ++failed;
    if (r.ready) {
        event_pool.push_back(r.ready);
        r.ready = nullptr;
    }
}

hipEvent_t Server::take_event_locked()
{
    if (!event_pool.empty()) {
        hipEvent_t e = event_pool.back();
        event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return e;
}

// Streams, events and the arena: everything create made, whether or not
// create finished (null handles are skipped).
void Server::release_resources()
{
    for (auto &sl : slots) {
        if (sl.st) (void)hipStreamSynchronize(sl.st);
        if (sl.done) (void)hipEventDestroy(sl.done);
        if (sl.st) (void)hipStreamDestroy(sl.st);
        sl.st = nullptr;
        sl.done = nullptr;
    }
    for (auto &kv : reqs)
        if (kv.second.ready) (void)hipEventDestroy(kv.second.ready);
    for (hipEvent_t e : event_pool) (void)hipEventDestroy(e);
    event_pool.clear();
    if (arena_mem) (void)hipFree(arena_mem);
    arena_mem = nullptr;
}

static int64_t footprint_of(const IJob &j)
{
    int64_t f = 4 * (j.m * j.k + j.k * j.n + j.m * j.n) + 2048; // operands, tables
    if (j.path == FF_PATH_INT8 && j.S > 0) {
        const I8Tile &t = i8_tile(i8_default_tile(j.S));
        // digit planes of the biggest tiling any batch may use (128-row tiles)
        const int64_t KP = round_up(std::max<int64_t>(j.k, 1), I8_BK);
        f += (int64_t)j.S * (round_up(j.m, std::max(t.bm(), 256)) +
                             round_up(j.n, std::max(t.bn(), 256))) * KP;
    } else if (j.path == FF_PATH_FP64) {
        // packed double operands (row tiles of at most 256)
        const int64_t KP = round_up(std::max<int64_t>(j.k, 1), F64_BK);
        f += (round_up(j.m, 256) + round_up(j.n, 256)) * KP * 8;
    }
    return align256(f);
}

bool Server::retire_locked()
{
    bool any = false;
    for (auto it = inflight.begin(); it != inflight.end();) {
        Slot &s = slots[it->first];
        hipError_t q = hipEventQuery(s.done);
        if (q == hipErrorNotReady) {
            ++it;
            continue;
        }
        const double t = now_s();
        const int status = q == hipSuccess ? FF_OK : FF_EHIP;
        for (uint64_t id : it->second.ids) {
            Request &r = reqs[id];
            finish_locked(r, status, t);
            lat_ms.push_back((t - r.t_submit) * 1e3);
            ops += 2.0 * (double)r.job.m * (double)r.job.n * (double)r.job.k;
            ++completed;
            --running_reqs;
        }
        t_last = t;
        if (it->second.arena_off >= 0) arena.release(it->second.arena_off);
        in_use -= it->second.footprint;
        s.busy = false;
        it = inflight.erase(it);
        any = true;
    }
    if (any) cv_done.notify_all();
    return any;
}

bool Server::admit_locked()
{
    bool launched = false;
    while (!queue.empty()) {
        int slot = -1;
        for (size_t i = 0; i < slots.size(); ++i)
            if (!slots[i].busy) { slot = (int)i; break; }
        if (slot < 0) break;
        // gather requests that fit, in arrival order
        std::vector<uint64_t> pick;
        std::vector<IJob> jobs;
        int64_t fp = 0;
        int Smax = 1;
        int path = -1;
        for (auto it = queue.begin(); it != queue.end() && (int)pick.size() < max_batch;) {
            Request &r = reqs[*it];
            if (path >= 0 && r.job.path != path) { ++it; continue; }
            if (in_use + fp + r.footprint > budget) { ++it; continue; }
            path = r.job.path;
            fp += r.footprint;
            Smax = std::max(Smax, r.job.S);
            jobs.push_back(r.job);
            pick.push_back(*it);
            it = queue.erase(it);
        }
        if (pick.empty()) break;
        Inflight f;
        f.slot = slot;
        f.ids = pick;
        f.footprint = fp;
        int tile;
        if (path == FF_PATH_INT8) {
            // the autotuner's choice for the batch's largest product, as for
            // ff_fgemm_batched
            int64_t bm = 1, bn = 1, bk = 1;
            for (const IJob &j : jobs)
                if (j.m * j.n * j.k > bm * bn * bk) { bm = j.m; bn = j.n; bk = j.k; }
            tile = tuned_i8_tile(Smax, bm, bn, bk);
            if (tile < 0) tile = i8_default_tile(Smax);
        } else {
            tile = choose_f64_tile();
        }
        int rc = prep_batch(jobs, path, tile, &f.prep);
        if (rc == FF_OK && !arena.alloc(std::max<int64_t>(f.prep.ws_bytes, 256), &f.arena_off)) {
            // fragmented arena: put the requests back (in order) and wait for
            // in-flight batches to return memory
            for (auto r = pick.rbegin(); r != pick.rend(); ++r) queue.push_front(*r);
            break;
        }
        Slot &s = slots[slot];
        // the batch starts after the writes its requests were submitted behind
        for (uint64_t id : pick) {
            const Request &r = reqs[id];
            if (rc == FF_OK && r.ready && hipStreamWaitEvent(s.st, r.ready, 0) != hipSuccess)
                rc = fail(FF_EHIP, "hipStreamWaitEvent failed");
        }
        if (rc == FF_OK) rc = upload_batch(f.prep, arena_mem + f.arena_off, s.st, false);
        unsigned *ctr = nullptr;
        if (rc == FF_OK) rc = counter_buffer(s.st, &ctr);
        if (rc == FF_OK) rc = launch_batch(f.prep, ctr, s.st, 1);
        for (const IJob &j : f.prep.singles)
            if (rc == FF_OK) rc = run_single_job(j, opts, s.st);
        if (rc == FF_OK && hipEventRecord(s.done, s.st) != hipSuccess) rc = FF_EHIP;
        if (rc != FF_OK) {
            // kernels already enqueued may still use the batch's range
            (void)hipStreamSynchronize(s.st);
            (void)hipGetLastError();
            const double t = now_s();
            for (uint64_t id : pick) finish_locked(reqs[id], rc, t);
            if (f.arena_off >= 0) arena.release(f.arena_off);
            cv_done.notify_all();
            continue;
        }
        for (uint64_t id : pick) reqs[id].state = 1;
        ++batches;
        max_batch_seen = std::max<int64_t>(max_batch_seen, (int64_t)pick.size());
        if (path == FF_PATH_INT8) last_tile = tile;
        running_reqs += (int64_t)pick.size();
        max_running = std::max(max_running, running_reqs);
        in_use += fp;
        s.busy = true;
        inflight.emplace(slot, std::move(f));
        launched = true;
    }
    return launched;
}

void Server::run()
{
    (void)hipSetDevice(device);
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
        retire_locked();
        admit_locked();
        if (stop && queue.empty() && inflight.empty()) break;
        if (inflight.empty())
            cv_work.wait(lk, [&] { return stop || !queue.empty(); });
        else
            cv_work.wait_for(lk, std::chrono::microseconds(20));
    }
}

} // namespace ff

using namespace ff;

extern "C" {

int ff_server_create(int64_t hbm_budget_bytes, const ff_opts *opts, void **server)
{
    if (!server) return fail(FF_EINVAL, "server is null");
    if (hbm_budget_bytes < 4096) return fail(FF_EINVAL, "budget too small");
    int rc = check_device();
    if (rc) return rc;
    Server *s = new Server();
    auto undo = [s](int status, const std::string &msg) {
        (void)hipGetLastError();
        s->release_resources();
        delete s;
        return fail(status, msg);
    };
    s->opts = opts ? *opts : default_opts();
    s->opts.winograd_levels = 0;
    s->budget = hbm_budget_bytes;
    if (hipGetDevice(&s->device) != hipSuccess) return undo(FF_EHIP, "hipGetDevice failed");
    if (hipMalloc(&s->arena_mem, hbm_budget_bytes) != hipSuccess) {
        s->arena_mem = nullptr;
        return undo(FF_ENOMEM, "server arena allocation of " +
                                   std::to_string(hbm_budget_bytes) + " bytes failed");
    }
    s->arena.reset(hbm_budget_bytes);
    const int nslots = 4;
    s->slots.resize(nslots);
    for (auto &sl : s->slots) {
        if (hipStreamCreateWithFlags(&sl.st, hipStreamNonBlocking) != hipSuccess) {
            sl.st = nullptr;
            return undo(FF_EHIP, "stream creation failed");
        }
        if (hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess) {
            sl.done = nullptr;
            return undo(FF_EHIP, "event creation failed");
        }
    }
    s->worker = std::thread([s] { s->run(); });
    *server = s;
    return FF_OK;
}

int ff_server_submit(void *server, const ff_job *job, uint64_t *id)
{
    if (!server || !job || !id) return fail(FF_EINVAL, "null argument");
    Server *s = (Server *)server;
    IJob j;
    int rc = job_from_abi(*job, s->opts, &j);
    if (rc) return rc;
    Request r;
    r.job = j;
    r.footprint = footprint_of(j);
    if (r.footprint > s->budget)
        return fail(FF_EBUSY, "request footprint " + std::to_string(r.footprint) +
                                  " exceeds the server budget");
    std::lock_guard<std::mutex> lk(s->mu);
    r.ready = s->take_event_locked();
    if (!r.ready) return fail(FF_EHIP, "event creation failed");
    if (hipEventRecord(r.ready, stream_of(&s->opts)) != hipSuccess) {
        (void)hipGetLastError();
        s->event_pool.push_back(r.ready);
        return fail(FF_EHIP, "hipEventRecord on the submitting stream failed");
    }
    r.t_submit = now_s();
    if (s->t_first < 0) s->t_first = r.t_submit;
    ++s->submitted;
    const uint64_t rid = s->next_id++;
    s->reqs.emplace(rid, r);
    s->queue.push_back(rid);
    *id = rid;
    s->cv_work.notify_one();
    return FF_OK;
}

int ff_server_poll(void *server, uint64_t id, int *done)
{
    if (!server || !done) return fail(FF_EINVAL, "null argument");
    Server *s = (Server *)server;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(id);
    if (it == s->reqs.end()) return fail(FF_ENOTFOUND, "unknown request id");
    *done = it->second.state >= 2;
    if (it->second.state == 3) return fail(it->second.status, "request failed");
    return FF_OK;
}

int ff_server_wait(void *server, uint64_t id)
{
    if (!server) return fail(FF_EINVAL, "null argument");
    Server *s = (Server *)server;
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(id);
    if (it == s->reqs.end()) return fail(FF_ENOTFOUND, "unknown request id");
    s->cv_done.wait(lk, [&] { return it->second.state >= 2; });
    if (it->second.state == 3) return fail(it->second.status, "request failed");
    return FF_OK;
}

int ff_server_stats(void *server, double *p50_ms, double *p99_ms, double *gops,
                    int64_t *completed, int64_t *max_inflight)
{
    if (!server) return fail(FF_EINVAL, "null argument");
    Server *s = (Server *)server;
    std::lock_guard<std::mutex> lk(s->mu);
    std::vector<double> l = s->lat_ms;
    std::sort(l.begin(), l.end());
    auto pct = [&](double q) {
        if (l.empty()) return 0.0;
        const double pos = q * (double)(l.size() - 1);
        const size_t i = (size_t)pos;
        const double f = pos - (double)i;
        return i + 1 < l.size() ? l[i] * (1 - f) + l[i + 1] * f : l[i];
    };
    if (p50_ms) *p50_ms = pct(0.50);
    if (p99_ms) *p99_ms = pct(0.99);
    if (gops) *gops = (s->t_last > s->t_first && s->t_first >= 0)
                          ? s->ops / (s->t_last - s->t_first) / 1e9 : 0.0;
    if (completed) *completed = s->completed;
    if (max_inflight) *max_inflight = s->max_running;
    return FF_OK;
}

int ff_server_query(void *server, ff_server_info *out)
{
    if (!server || !out) return fail(FF_EINVAL, "null argument");
    Server *s = (Server *)server;
    std::lock_guard<std::mutex> lk(s->mu);
    std::memset(out, 0, sizeof(*out));
    out->submitted = s->submitted;
    out->completed = s->completed;
    out->failed = s->failed;
    out->queued = (int64_t)s->queue.size();
    out->running = s->running_reqs;
    out->batches = s->batches;
    out->max_batch_requests = s->max_batch_seen;
    out->max_inflight = s->max_running;
    out->hbm_budget = s->budget;
    out->hbm_in_use = s->in_use;
    out->last_i8_tile = s->last_tile;
    out->stream_slots = (int)s->slots.size();
    return FF_OK;
}

int ff_server_destroy(void *server)
{
    if (!server) return fail(FF_EINVAL, "null argument");
    Server *s = (Server *)server;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        s->cv_work.notify_all();
    }
    s->worker.join();
    s->release_resources();
    delete s;
    return FF_OK;
}

} // extern "C"
