// Served form of libfsz.so: a request loop with admission by device memory
// and continuous batching into the batched launch (fsz_batch_async).
//
// One worker thread per server owns the schedule:
//   arrived requests (arrival time passed) -> admission in arrival order when
//   the output reservation fits in the arena -> folded, up to
//   max_jobs_per_round at a time, into a batched launch on the next idle
//   stream -> completion when that stream's event has fired.
// Rounds on different streams overlap on the device, so requests that
// arrive while a round runs start at once on another stream instead of
// waiting for it.  The worker only enqueues and polls; all compression
// work is the batched kernels'.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <queue>
#include <set>
#include <thread>
#include <vector>

#include "fsz_arena.h"
#include "fsz_internal.h"

using namespace fsz;

namespace {

bool ok(hipError_t e) { return e == hipSuccess; }

uint64_t clock_ns()
{
    return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

struct ReqRec {
    fsz_request r;
    uint64_t seq = 0;  // submission order (ties of equal arrival times)
    uint64_t off = 0, bytes = 0, admit_ns = 0;
};

struct LaterArrival {
    bool operator()(const ReqRec &a, const ReqRec &b) const
    {
        return a.r.arrival_ns != b.r.arrival_ns ? a.r.arrival_ns > b.r.arrival_ns : a.seq > b.seq;
    }
};

// One stream and the round it runs.
struct RoundSlot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    fsz_result *d_res = nullptr;
    fsz_result *h_res = nullptr;  // pinned copy, valid once `done` fired
    size_t cap = 0;
    std::vector<ReqRec> jobs;
    std::vector<fsz_job> jv;
    bool busy = false;
    uint64_t launch_ns = 0;
};

// Output bytes reserved for a request: the worst-case stream for a
// compression, the float field for a decompression.
uint64_t reserve_bytes(const fsz_request &r)
{
    return r.op == FSZ_OP_COMPRESS ? (uint64_t)fsz_compressed_bound(r.n) : 4ull * r.n;
}

fsz_status check_request(const fsz_request &r)
{
    if (r.op == FSZ_OP_COMPRESS) {
        if (!valid_bound(r.mode, r.value) || (r.n > 0 && !r.d_src) || !aligned(r.d_src, 4))
            return FSZ_ERR_INVALID_ARG;
        return FSZ_OK;
    }
    if (r.op == FSZ_OP_DECOMPRESS) {
        if (!r.d_src || !aligned(r.d_src, 4)) return FSZ_ERR_INVALID_ARG;
        if (r.src_size < (size_t)kHeaderBytes) return FSZ_ERR_CORRUPT;
        return FSZ_OK;
    }
    return FSZ_ERR_INVALID_ARG;
}

}  // namespace

struct fsz_server {
    fsz_server_config cfg{};
    int device = 0;
    char *base = nullptr;  // device arena
    Arena arena;
    std::set<uint64_t> held;  // completed outputs not yet released (arena offsets)
    std::mutex arena_mu;

    std::vector<RoundSlot> slots;
    std::thread worker;

    std::mutex mu;  // inbox, stop, stats
    std::condition_variable cv;
    std::vector<ReqRec> inbox;
    uint64_t next_seq = 0;
    bool stop = false;
    fsz_server_stats stats{};

    std::mutex cmu;  // completions
    std::condition_variable ccv;
    std::deque<fsz_completion> done;

    // worker-only state
    std::priority_queue<ReqRec, std::vector<ReqRec>, LaterArrival> future;
    std::deque<ReqRec> waiting, ready;
};

namespace {

void push_completions(fsz_server *s, std::vector<fsz_completion> &cs)
{
    if (cs.empty()) return;
    {
        std::lock_guard<std::mutex> g(s->cmu);
        for (auto &c : cs) s->done.push_back(c);
    }
    {
        std::lock_guard<std::mutex> g(s->mu);
        s->stats.completed += cs.size();
    }
    s->ccv.notify_all();
    cs.clear();
}

fsz_completion make_completion(const ReqRec &q, uint32_t status, uint64_t size, void *out, uint64_t launch,
                               uint64_t complete)
{
    fsz_completion c{};
    c.tag = q.r.tag;
    c.status = status;
    c.op = (uint32_t)q.r.op;
    c.size = size;
    c.d_out = out;
    c.arrival_ns = q.r.arrival_ns;
    c.admit_ns = q.admit_ns;
    c.launch_ns = launch;
    c.complete_ns = complete;
    return c;
}

// Enqueue one round of admitted requests on an idle slot.
void launch_round(fsz_server *s, RoundSlot &slot, std::vector<fsz_completion> &failed)
{
    const size_t k = std::min(s->ready.size(), (size_t)s->cfg.max_jobs_per_round);
    slot.jobs.assign(s->ready.begin(), s->ready.begin() + (long)k);
    s->ready.erase(s->ready.begin(), s->ready.begin() + (long)k);
    const uint64_t t_launch = clock_ns();
    auto fail_all = [&](uint32_t st) {
        std::lock_guard<std::mutex> g(s->arena_mu);
        for (auto &q : slot.jobs) {
            s->arena.release(q.off);
            failed.push_back(make_completion(q, st, 0, nullptr, t_launch, clock_ns()));
        }
        slot.jobs.clear();
    };
    if (k > slot.cap) {
        if (slot.d_res) (void)hipFree(slot.d_res);
        if (slot.h_res) (void)hipHostFree(slot.h_res);
        slot.d_res = nullptr;
        slot.h_res = nullptr;
        slot.cap = 0;
        size_t c = 64;
        while (c < k) c *= 2;
        if (!ok(hipMalloc(&slot.d_res, c * sizeof(fsz_result))) ||
            !ok(hipHostMalloc(&slot.h_res, c * sizeof(fsz_result), hipHostMallocDefault))) {
            fail_all(FSZ_ERR_DEVICE);
            return;
        }
        slot.cap = c;
    }
    slot.jv.resize(k);
    for (size_t i = 0; i < k; i++) {
        const fsz_request &r = slot.jobs[i].r;
        fsz_job &j = slot.jv[i];
        j.op = r.op;
        j.d_src = r.d_src;
        j.src_size = r.src_size;
        j.d_dst = s->base + slot.jobs[i].off;
        j.dst_capacity = r.op == FSZ_OP_COMPRESS ? slot.jobs[i].bytes : 0;
        j.n = r.n;
        j.mode = r.mode;
        j.value = r.value;
        j.d_result = slot.d_res + i;
    }
    // results the kernels do not write read back as a device error
    if (!ok(hipMemsetAsync(slot.d_res, 0xFF, k * sizeof(fsz_result), slot.stream))) {
        fail_all(FSZ_ERR_DEVICE);
        return;
    }
    const fsz_status st = fsz_batch_async(slot.jv.data(), k, &s->cfg.tuning, slot.stream);
    if (st != FSZ_OK) {
        fail_all(st);
        return;
    }
    if (!ok(hipMemcpyAsync(slot.h_res, slot.d_res, k * sizeof(fsz_result), hipMemcpyDeviceToHost, slot.stream)) ||
        !ok(hipEventRecord(slot.done, slot.stream))) {
        // the batch is enqueued: wait for it before its outputs are reused
        (void)hipStreamSynchronize(slot.stream);
        fail_all(FSZ_ERR_DEVICE);
        return;
    }
    slot.busy = true;
    slot.launch_ns = t_launch;
    uint64_t busy = 0;
    for (auto &o : s->slots) busy += o.busy ? 1 : 0;
    std::lock_guard<std::mutex> g(s->mu);
    s->stats.rounds++;
    s->stats.max_jobs_in_round = std::max<uint64_t>(s->stats.max_jobs_in_round, k);
    s->stats.max_rounds_overlapping = std::max<uint64_t>(s->stats.max_rounds_overlapping, busy);
}

void finish_round(fsz_server *s, RoundSlot &slot, std::vector<fsz_completion> &out)
{
    const uint64_t t = clock_ns();
    std::lock_guard<std::mutex> g(s->arena_mu);
    for (size_t i = 0; i < slot.jobs.size(); i++) {
        const ReqRec &q = slot.jobs[i];
        const fsz_result &r = slot.h_res[i];
        uint32_t st = r.status;
        if (st > (uint32_t)FSZ_ERR_EB_TOO_LARGE) st = FSZ_ERR_DEVICE;  // never written
        void *d_out = nullptr;
        if (st == FSZ_OK && !s->cfg.auto_release) {
            d_out = s->base + q.off;
            s->held.insert(q.off);
        } else {
            s->arena.release(q.off);
        }
        out.push_back(make_completion(q, st, st == FSZ_OK ? r.size : 0, d_out, slot.launch_ns, t));
    }
    slot.jobs.clear();
    slot.busy = false;
}

void worker_main(fsz_server *s)
{
    (void)hipSetDevice(s->device);
    std::vector<fsz_completion> out;
    for (;;) {
        bool progress = false;
        bool stopping;
        {
            std::lock_guard<std::mutex> g(s->mu);
            for (auto &q : s->inbox) s->future.push(q);
            s->inbox.clear();
            stopping = s->stop;
        }
        const uint64_t now = clock_ns();
        while (!s->future.empty() && s->future.top().r.arrival_ns <= now) {
            s->waiting.push_back(s->future.top());
            s->future.pop();
            progress = true;
        }
        // admission in arrival order
        while (!s->waiting.empty()) {
            ReqRec &q = s->waiting.front();
            const uint64_t need = reserve_bytes(q.r);
            uint64_t off = 0;
            bool fits;
            {
                std::lock_guard<std::mutex> g(s->arena_mu);
                if (!s->arena.fits_ever(need)) {
                    const uint64_t t = clock_ns();
                    q.admit_ns = t;
                    out.push_back(make_completion(q, FSZ_ERR_CAPACITY, 0, nullptr, t, t));
                    s->waiting.pop_front();
                    progress = true;
                    continue;
                }
                fits = s->arena.alloc(need, &off);
            }
            if (!fits) break;
            q.off = off;
            q.bytes = Arena::round_up(need);
            q.admit_ns = clock_ns();
            s->ready.push_back(q);
            s->waiting.pop_front();
            progress = true;
        }
        // completions first: they free slots for the launches below
        bool any_busy = false;
        for (auto &slot : s->slots) {
            if (slot.busy && hipEventQuery(slot.done) == hipSuccess) {
                finish_round(s, slot, out);
                progress = true;
            }
            any_busy = any_busy || slot.busy;
        }
        for (auto &slot : s->slots) {
            if (s->ready.empty()) break;
            if (slot.busy) continue;
            launch_round(s, slot, out);
            progress = true;
            any_busy = any_busy || slot.busy;
        }
        push_completions(s, out);
        if (progress) continue;
        if (any_busy) {
            std::this_thread::yield();  // rounds in flight: keep polling their events
            continue;
        }
        if (stopping && s->future.empty() && s->ready.empty()) {
            if (s->waiting.empty()) break;
            // shutting down with requests blocked behind unreleased outputs:
            // the caller is done with them
            std::lock_guard<std::mutex> g(s->arena_mu);
            if (s->held.empty()) break;  // cannot happen: nothing else holds the arena
            for (uint64_t off : s->held) s->arena.release(off);
            s->held.clear();
            continue;
        }
        std::unique_lock<std::mutex> g(s->mu);
        if (!s->inbox.empty() || s->stop != stopping) continue;
        if (!s->future.empty()) {
            const uint64_t wake = s->future.top().r.arrival_ns;
            const uint64_t t = clock_ns();
            if (wake > t) {
                // sleep until the next arrival, but not past 1 ms: the kernel's
                // wake-up slack would otherwise add to the arrival's latency
                const uint64_t d = std::min<uint64_t>(wake - t, 1000000);
                if (d > 200000) s->cv.wait_for(g, std::chrono::nanoseconds(d - 100000));
            }
        } else if (!s->waiting.empty()) {
            s->cv.wait_for(g, std::chrono::milliseconds(1));  // memory held by the caller
        } else {
            s->cv.wait_for(g, std::chrono::milliseconds(50));
        }
    }
    push_completions(s, out);
}

void free_server(fsz_server *s)
{
    for (auto &slot : s->slots) {
        if (slot.stream) (void)hipStreamSynchronize(slot.stream);
        if (slot.done) (void)hipEventDestroy(slot.done);
        if (slot.stream) (void)hipStreamDestroy(slot.stream);
        if (slot.d_res) (void)hipFree(slot.d_res);
        if (slot.h_res) (void)hipHostFree(slot.h_res);
    }
    if (s->base) (void)hipFree(s->base);
    delete s;
}

}  // namespace

extern "C" {

uint64_t fsz_server_now_ns(void) { return clock_ns(); }

fsz_status fsz_server_create(const fsz_server_config *cfg, fsz_server **server)
{
    if (!cfg || !server) return FSZ_ERR_INVALID_ARG;
    *server = nullptr;
    if (cfg->hbm_budget == 0 || cfg->max_jobs_per_round < 1 || cfg->max_jobs_per_round > 65536 ||
        cfg->rounds_in_flight < 1 || cfg->rounds_in_flight > 16)
        return FSZ_ERR_INVALID_ARG;
    fsz_server_config c = *cfg;
    if (c.tuning.waves_per_group == 0 && c.tuning.groups_per_cu == 0) c.tuning = fsz_tuning{4, 0};
    BatchShape shape;
    shape.waves = c.tuning.waves_per_group;
    shape.groups_per_cu = c.tuning.groups_per_cu;
    if (!batch_shape_supported(shape)) return FSZ_ERR_INVALID_ARG;
    auto *s = new fsz_server();
    s->cfg = c;
    bool good = ok(hipGetDevice(&s->device)) && ok(hipMalloc(&s->base, c.hbm_budget));
    s->arena.reset(c.hbm_budget);
    s->slots.resize((size_t)c.rounds_in_flight);
    for (auto &slot : s->slots) {
        good = good && ok(hipStreamCreateWithFlags(&slot.stream, hipStreamNonBlocking)) &&
               ok(hipEventCreateWithFlags(&slot.done, hipEventDisableTiming));
    }
    // Everything a round can need is allocated now: growing it later would
    // free device memory, which waits for every stream of the device.
    // Outputs of one round fit in the arena, and every output reserves at
    // least 4 bytes per element, so a round covers at most budget / 4
    // elements.
    const uint64_t jobs = (uint64_t)c.max_jobs_per_round;
    const uint64_t elems = c.hbm_budget / 4;
    const uint64_t chunks = elems / ((uint64_t)kTile * kTilesPerWave * (uint64_t)c.tuning.waves_per_group) + jobs;
    const uint64_t segs = elems / kSegElems + jobs;
    for (auto &slot : s->slots) {
        if (!good) break;
        size_t cap = 64;
        while (cap < jobs) cap *= 2;
        good = reserve_batch(slot.stream, jobs, chunks, segs) &&
               ok(hipMalloc(&slot.d_res, cap * sizeof(fsz_result))) &&
               ok(hipHostMalloc(&slot.h_res, cap * sizeof(fsz_result), hipHostMallocDefault));
        if (good) slot.cap = cap;
    }
    if (!good) {
        free_server(s);
        return FSZ_ERR_DEVICE;
    }
    s->worker = std::thread(worker_main, s);
    *server = s;
    return FSZ_OK;
}

fsz_status fsz_server_submit(fsz_server *server, const fsz_request *reqs, size_t count)
{
    if (!server || (count > 0 && !reqs)) return FSZ_ERR_INVALID_ARG;
    for (size_t k = 0; k < count; k++) {
        const fsz_status st = check_request(reqs[k]);
        if (st != FSZ_OK) return st;
    }
    {
        std::lock_guard<std::mutex> g(server->mu);
        if (server->stop) return FSZ_ERR_INVALID_ARG;
        for (size_t k = 0; k < count; k++) {
            ReqRec q;
            q.r = reqs[k];
            q.seq = server->next_seq++;
            server->inbox.push_back(q);
        }
        server->stats.submitted += count;
    }
    server->cv.notify_all();
    return FSZ_OK;
}

size_t fsz_server_poll(fsz_server *server, fsz_completion *out, size_t max, int wait_ms)
{
    if (!server || !out || max == 0) return 0;
    std::unique_lock<std::mutex> g(server->cmu);
    if (server->done.empty() && wait_ms > 0)
        server->ccv.wait_for(g, std::chrono::milliseconds(wait_ms), [&] { return !server->done.empty(); });
    size_t k = 0;
    while (k < max && !server->done.empty()) {
        out[k++] = server->done.front();
        server->done.pop_front();
    }
    return k;
}

fsz_status fsz_server_release(fsz_server *server, void *d_out)
{
    if (!server || !d_out) return FSZ_ERR_INVALID_ARG;
    const char *p = static_cast<const char *>(d_out);
    if (p < server->base || p >= server->base + server->arena.size()) return FSZ_ERR_INVALID_ARG;
    const uint64_t off = (uint64_t)(p - server->base);
    {
        std::lock_guard<std::mutex> g(server->arena_mu);
        if (!server->held.count(off)) return FSZ_ERR_INVALID_ARG;
        server->held.erase(off);
        server->arena.release(off);
    }
    server->cv.notify_all();
    return FSZ_OK;
}

fsz_status fsz_server_get_stats(fsz_server *server, fsz_server_stats *out)
{
    if (!server || !out) return FSZ_ERR_INVALID_ARG;
    fsz_server_stats st;
    {
        std::lock_guard<std::mutex> g(server->mu);
        st = server->stats;
    }
    {
        std::lock_guard<std::mutex> g(server->arena_mu);
        st.hbm_in_use = server->arena.used();
        st.hbm_peak = server->arena.peak();
    }
    *out = st;
    return FSZ_OK;
}

void fsz_server_destroy(fsz_server *server)
{
    if (!server) return;
    {
        std::lock_guard<std::mutex> g(server->mu);
        server->stop = true;
    }
    server->cv.notify_all();
    if (server->worker.joinable()) server->worker.join();
    free_server(server);
}

}  // extern "C"
