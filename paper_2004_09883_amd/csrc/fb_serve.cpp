// fb_serve.cpp -- the serving form: a request loop that runs spectral-block
// requests of mixed shapes and dtypes on one GPU with continuous batching.
//
// A worker thread owns the device side.  Submitted requests wait in a queue;
// the worker admits the next one (the oldest, or under FB_SERVE_DEADLINE the
// one with the earliest arrival plus estimated service time) whenever a
// stream slot is free and its bytes fit in the HBM budget, so requests that arrive while others
// are on the GPU start as soon as a slot and memory free up and their work
// overlaps on the device (one HIP stream per slot).  Plans are cached per
// (shape, dtype) and device buffers are pooled by size, so both stay
// resident across requests; pooled memory counts against the budget.
//
// One request: generate the seeded input grid on the device, forward 3D FFT
// in place, then for t = 1..T the fused evolve + inverse + checksum into a
// second grid, copy the T checksums (and, on request, the final grid) to
// pinned host memory, record an event.  The worker polls the events and
// stamps the completion time.  The kernels and the order of operations of a
// request do not depend on what else runs, so a result is bitwise the same
// alone and in a mix.
#include <hip/hip_runtime.h>

#include <stdio.h>
#include <string.h>

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <tuple>
#include <vector>

#include "fb.h"
#include "fb_internal.hpp"

namespace {

double now_s()
{
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

uint64_t splitmix64_at(uint64_t seed, uint64_t c)
{
    uint64_t z = seed + (c + 1ull) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

struct Pending {
    fb_request req;
    int64_t id;
    double t_arrival;
};

struct Slot {
    bool busy = false;
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    int64_t id = -1;
    fb_request req{};
    double t_arrival = 0, t_admit = 0;
    void *u0 = nullptr, *x = nullptr;      // device grids: the spectrum, the output grids of a chunk of steps
    double *sums_dev = nullptr;            // device checksums
    size_t grid_bytes = 0, x_bytes = 0, sums_bytes = 0;
    size_t charged = 0;                    // bytes charged to the budget
    double *sums_host = nullptr;           // pinned, FB_SERVE_MAX_STEPS checksums, owned by the slot
    void *grid_host = nullptr;             // pinned (when the final grid is wanted)
};

struct Done {
    fb_result res;
    std::vector<double> sums;
    std::vector<char> grid;
};

}  // namespace

struct fb_server {
    size_t budget;
    int device;
    std::vector<Slot> slots;
    // plans and pool belong to the worker thread (and to fb_server_destroy
    // after the worker has joined); the figures fb_server_stats reports are
    // atomics, so no other thread reads what the worker writes unguarded
    std::map<std::tuple<int64_t, int64_t, int64_t, int>, fb_plan *> plans;
    std::multimap<size_t, void *> pool;    // free device buffers by size
    std::atomic<size_t> bytes_allocated{0};   // pooled + in use (device)
    std::atomic<size_t> peak_allocated{0};
    std::atomic<int> plans_cached{0};
    std::mutex mu;
    std::condition_variable cv;
    std::deque<Pending> queue;
    std::deque<Done> done;
    std::thread worker;
    std::atomic<bool> stop{false};
    int64_t next_id = 0;
    int64_t in_flight = 0;
    std::atomic<int> policy{FB_SERVE_FIFO};
    int last_error = FB_OK;
    std::string last_msg;
    std::atomic<int> max_concurrent{0};
};

namespace {

size_t esize_of(int dtype) { return dtype == FB_C128 ? 16 : 8; }

// Steps computed together from one read of the spectrum (fb_spectral_steps):
// a request holds this many output grids.
constexpr int kChunk = 8;
int chunk_of(int steps) { return steps < kChunk ? steps : kChunk; }

size_t sums_bytes_of(int steps) { return 256 * ((size_t)(16 * steps + 255) / 256); }

// Device bytes a request holds while admitted: the spectrum, the output
// grids of one chunk of steps and its checksums.
size_t request_bytes(const fb_request &r)
{
    const size_t n = (size_t)(r.nx * r.ny * r.nz);
    return (1 + (size_t)chunk_of(r.steps)) * n * esize_of(r.dtype) + sums_bytes_of(r.steps);
}

// Estimated service time of a request alone on the device: the grids its
// passes move (input generated in the first forward pass: 5 grids for the
// forward transform; one read of the spectrum per chunk of steps; 5 grids per
// step) at a nominal 5 TB/s.
double service_estimate_s(const fb_request &r)
{
    const double grid = (double)(r.nx * r.ny * r.nz) * (double)esize_of(r.dtype);
    const double chunks = (double)((r.steps + kChunk - 1) / kChunk);
    return grid * (5.0 + chunks + 5.0 * r.steps) / 5e12;
}

// Index of the queued request to admit next (the queue is not empty).
size_t next_index(fb_server *s)
{
    if (s->policy.load() != FB_SERVE_DEADLINE) return 0;
    size_t best = 0;
    double key = 0;
    for (size_t i = 0; i < s->queue.size(); i++) {
        const double k = s->queue[i].t_arrival + service_estimate_s(s->queue[i].req);
        if (i == 0 || k < key) {
            best = i;
            key = k;
        }
    }
    return best;
}

void *pool_get(fb_server *s, size_t bytes, hipError_t &e)
{
    auto it = s->pool.find(bytes);
    if (it != s->pool.end()) {
        void *p = it->second;
        s->pool.erase(it);
        return p;
    }
    // make room: give back pooled buffers of other sizes first
    while (s->bytes_allocated.load() + bytes > s->budget && !s->pool.empty()) {
        auto big = std::prev(s->pool.end());
        (void)hipFree(big->second);
        s->bytes_allocated -= big->first;
        s->pool.erase(big);
    }
    void *p = nullptr;
    e = hipMalloc(&p, bytes);
    if (e != hipSuccess) return nullptr;
    const size_t now = (s->bytes_allocated += bytes);
    if (now > s->peak_allocated.load()) s->peak_allocated.store(now);   // only the worker writes it
    return p;
}

void pool_put(fb_server *s, size_t bytes, void *p)
{
    if (p) s->pool.emplace(bytes, p);
}

// Admission test: the device bytes in use by admitted requests plus what r
// needs must fit in the budget (pooled free buffers can always be released).
bool fits(fb_server *s, const fb_request &r)
{
    size_t in_use = s->bytes_allocated.load();
    for (auto &kv : s->pool) in_use -= kv.first;
    return in_use + request_bytes(r) <= s->budget;
}

fb_plan *plan_for(fb_server *s, const fb_request &r)
{
    auto key = std::make_tuple(r.nx, r.ny, r.nz, r.dtype);
    auto it = s->plans.find(key);
    if (it != s->plans.end()) return it->second;
    fb_plan *p = fb_fft3d_plan(r.nx, r.ny, r.nz, r.dtype);
    if (p) {
        // the concurrent requests' grids together exceed the last-level cache:
        // every pass streams (measured at 2000 req/s: end-to-end p50 16 ms,
        // p99 71 ms; with the non-temporal instances only for grids above
        // the cache size, p50 48 ms, p99 127 ms)
        fb::plan_set_nt_always(p, true);
        s->plans[key] = p;
        s->plans_cached.store((int)s->plans.size());
    }
    return p;
}

void finish(fb_server *s, Slot &sl, int status)
{
    Done d{};
    d.res.id = sl.id;
    d.res.status = status;
    d.res.nx = sl.req.nx;
    d.res.ny = sl.req.ny;
    d.res.nz = sl.req.nz;
    d.res.dtype = sl.req.dtype;
    d.res.steps = sl.req.steps;
    d.res.t_arrival = sl.t_arrival;
    d.res.t_admit = sl.t_admit;
    d.res.t_done = now_s();
    if (status == FB_OK) {
        d.sums.assign(sl.sums_host, sl.sums_host + 2 * sl.req.steps);
        if (sl.grid_host) {
            const char *g = (const char *)sl.grid_host;
            d.grid.assign(g, g + sl.grid_bytes);
        }
    }
    pool_put(s, sl.grid_bytes, sl.u0);
    pool_put(s, sl.x_bytes, sl.x);
    pool_put(s, sl.sums_bytes, sl.sums_dev);
    if (sl.grid_host) (void)hipHostFree(sl.grid_host);
    sl.u0 = sl.x = nullptr;
    sl.sums_dev = nullptr;
    sl.grid_host = nullptr;
    sl.busy = false;
    std::lock_guard<std::mutex> lk(s->mu);
    s->in_flight--;
    s->done.push_back(std::move(d));
}

// Enqueues the whole request on the slot's stream.
int launch(fb_server *s, Slot &sl)
{
    const fb_request &r = sl.req;
    fb_plan *p = plan_for(s, r);
    if (!p) return fb_last_error(nullptr);
    hipError_t e = hipSuccess;
    const int chunk = chunk_of(r.steps);
    sl.grid_bytes = (size_t)(r.nx * r.ny * r.nz) * esize_of(r.dtype);
    sl.x_bytes = (size_t)chunk * sl.grid_bytes;
    sl.sums_bytes = sums_bytes_of(r.steps);
    sl.u0 = pool_get(s, sl.grid_bytes, e);
    if (e == hipSuccess) sl.x = pool_get(s, sl.x_bytes, e);
    if (e == hipSuccess) sl.sums_dev = (double *)pool_get(s, sl.sums_bytes, e);
    if (e == hipSuccess && r.want_grid) e = hipHostMalloc(&sl.grid_host, sl.grid_bytes, hipHostMallocDefault);
    if (e != hipSuccess) return FB_ERR_OOM;
    const uint64_t seed = splitmix64_at(r.seed, (uint64_t)r.request_key);
    int rc = fb_fft3d_forward_uniform(p, seed, sl.u0, sl.stream);
    // steps t = 1..steps in chunks: each chunk reads the spectrum once
    double ts[kChunk];
    int last = 0;   // grid of the final step within the buffer
    for (int j0 = 0; !rc && j0 < r.steps; j0 += chunk) {
        const int k = r.steps - j0 < chunk ? r.steps - j0 : chunk;
        for (int i = 0; i < k; i++) ts[i] = (double)(j0 + i + 1);
        rc = fb_spectral_steps(p, sl.u0, sl.x, r.alpha, ts, k, sl.sums_dev + 2 * j0, sl.stream);
        last = k - 1;
    }
    if (rc) return rc;
    e = hipMemcpyAsync(sl.sums_host, sl.sums_dev, 16 * (size_t)r.steps, hipMemcpyDeviceToHost, sl.stream);
    if (e == hipSuccess && sl.grid_host)
        e = hipMemcpyAsync(sl.grid_host, (const char *)sl.x + (size_t)last * sl.grid_bytes, sl.grid_bytes,
                           hipMemcpyDeviceToHost, sl.stream);
    if (e == hipSuccess) e = hipEventRecord(sl.done, sl.stream);
    return e == hipSuccess ? FB_OK : FB_ERR_DEVICE;
}

void worker_loop(fb_server *s)
{
    (void)hipSetDevice(s->device);
    while (true) {
        bool idle = true;
        // completions
        for (Slot &sl : s->slots) {
            if (!sl.busy) continue;
            hipError_t q = hipEventQuery(sl.done);
            if (q == hipSuccess) {
                finish(s, sl, FB_OK);
                idle = false;
            } else if (q != hipErrorNotReady) {
                finish(s, sl, FB_ERR_DEVICE);
                idle = false;
            }
        }
        // admissions, in the order of the policy
        for (;;) {
            Pending head;
            size_t hi;
            {
                std::lock_guard<std::mutex> lk(s->mu);
                if (s->queue.empty()) break;
                hi = next_index(s);
                head = s->queue[hi];
            }
            Slot *free_slot = nullptr;
            for (Slot &sl : s->slots)
                if (!sl.busy) {
                    free_slot = &sl;
                    break;
                }
            if (!free_slot || !fits(s, head.req)) break;
            {
                std::lock_guard<std::mutex> lk(s->mu);
                s->queue.erase(s->queue.begin() + (std::ptrdiff_t)hi);   // only this thread removes entries
            }
            Slot &sl = *free_slot;
            sl.busy = true;
            sl.id = head.id;
            sl.req = head.req;
            sl.t_arrival = head.t_arrival;
            sl.t_admit = now_s();
            int busy = 0;
            for (Slot &o : s->slots) busy += o.busy ? 1 : 0;
            if (busy > s->max_concurrent.load()) s->max_concurrent.store(busy);   // only the worker writes it
            const int rc = launch(s, sl);
            if (rc != FB_OK) {
                (void)hipStreamSynchronize(sl.stream);
                finish(s, sl, rc);
            }
            idle = false;
        }
        if (s->stop.load()) {
            bool any = false;
            for (Slot &sl : s->slots) any = any || sl.busy;
            std::lock_guard<std::mutex> lk(s->mu);
            if (!any && s->queue.empty()) break;
        }
        if (idle) {
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv.wait_for(lk, std::chrono::microseconds(20));
        }
    }
}

}  // namespace

extern "C" {

fb_server *fb_server_create(size_t budget_bytes, int n_streams)
{
    if (n_streams < 1 || n_streams > 64 || budget_bytes < (1u << 20)) return nullptr;
    fb_server *s = new (std::nothrow) fb_server();
    if (!s) return nullptr;
    s->budget = budget_bytes;
    if (hipGetDevice(&s->device) != hipSuccess) {
        delete s;
        return nullptr;
    }
    s->slots.resize(n_streams);
    for (Slot &sl : s->slots) {
        if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess ||
            hipHostMalloc((void **)&sl.sums_host, 16 * FB_SERVE_MAX_STEPS, hipHostMallocDefault) != hipSuccess) {
            for (Slot &o : s->slots) {
                if (o.stream) (void)hipStreamDestroy(o.stream);
                if (o.done) (void)hipEventDestroy(o.done);
                if (o.sums_host) (void)hipHostFree(o.sums_host);
            }
            delete s;
            return nullptr;
        }
    }
    s->worker = std::thread(worker_loop, s);
    return s;
}

int64_t fb_server_submit(fb_server *s, const fb_request *r)
{
    if (!s || !r) return FB_ERR_INVALID_ARG;
    if (r->dtype != FB_C128 && r->dtype != FB_C64) return FB_ERR_DTYPE;
    if (r->steps < 1 || r->steps > FB_SERVE_MAX_STEPS || !(r->alpha >= 0)) return FB_ERR_INVALID_ARG;
    char tmp[128];
    if (fb_describe_shape(r->nx, r->ny, r->nz, r->dtype, tmp, sizeof tmp) < 0) return fb_last_error(nullptr);
    if (request_bytes(*r) > s->budget) return FB_ERR_BUDGET;
    Pending p;
    p.req = *r;
    p.t_arrival = now_s();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        p.id = s->next_id++;
        s->queue.push_back(p);
        s->in_flight++;
    }
    s->cv.notify_one();
    return p.id;
}

int fb_server_poll(fb_server *s, fb_result *out, double *sums, int sums_cap, void *grid, size_t grid_cap)
{
    if (!s || !out) return FB_ERR_INVALID_ARG;
    Done d;
    {
        // take the result out under the lock; copy it out after releasing
        // the lock, so a large final grid does not hold up the worker
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->done.empty()) return 0;
        d = std::move(s->done.front());
        s->done.pop_front();
    }
    *out = d.res;
    if (sums && sums_cap > 0) {
        const size_t n = d.sums.size() < (size_t)sums_cap ? d.sums.size() : (size_t)sums_cap;
        memcpy(sums, d.sums.data(), n * sizeof(double));
    }
    out->grid_bytes = (int64_t)d.grid.size();
    if (grid && !d.grid.empty() && grid_cap >= d.grid.size()) memcpy(grid, d.grid.data(), d.grid.size());
    return 1;
}

int64_t fb_server_in_flight(fb_server *s)
{
    if (!s) return FB_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    return s->in_flight;
}

int fb_server_set_policy(fb_server *s, int policy)
{
    if (!s || (policy != FB_SERVE_FIFO && policy != FB_SERVE_DEADLINE)) return FB_ERR_INVALID_ARG;
    s->policy.store(policy);
    return FB_OK;
}

int fb_server_stats(fb_server *s, fb_server_info *info)
{
    if (!s || !info) return FB_ERR_INVALID_ARG;
    info->budget = s->budget;
    info->bytes_allocated = s->bytes_allocated.load();
    info->peak_allocated = s->peak_allocated.load();
    info->plans_cached = s->plans_cached.load();
    info->max_concurrent = s->max_concurrent.load();
    std::lock_guard<std::mutex> lk(s->mu);
    info->queued = (int64_t)s->queue.size();
    return FB_OK;
}

void fb_server_destroy(fb_server *s)
{
    if (!s) return;
    s->stop.store(true);
    s->cv.notify_one();
    if (s->worker.joinable()) s->worker.join();
    for (Slot &sl : s->slots) {
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
        if (sl.done) (void)hipEventDestroy(sl.done);
        if (sl.sums_host) (void)hipHostFree(sl.sums_host);
    }
    for (auto &kv : s->pool) (void)hipFree(kv.second);
    for (auto &kv : s->plans) fb_fft3d_destroy(kv.second);
    delete s;
}

}  // extern "C"
