// Continuous-batching server of the truncated-multiplication library (see
// the tm_server_* declarations in include/tmul.h).
//
// A server owns one device memory pool, a few HIP streams and a number of
// request slots.  Requests carry host operand / result buffers.  They wait
// in arrival order; a request is admitted as soon as a slot is free and its
// device footprint (operands, result, guard, workspace) can be carved out of
// the pool, and then runs on the
// stream with the fewest requests in flight: operands in, tm_mul, result
// and guard out, completion event.  Polling retires finished requests,
// returns their memory and admits more, so requests that arrive while others
// run join the device as soon as memory frees up, and their work overlaps
// on the device through the streams.  A request that does not fit reserves
// the bytes it is waiting for, so smaller requests behind it can pass it
// only within the remaining space (no starvation of large requests).
#include <hip/hip_runtime.h>

#include <chrono>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <new>
#include <string>
#include <vector>

#include "tmul.h"

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

double now_s()
{
    using clk = std::chrono::steady_clock;
    return std::chrono::duration<double>(clk::now().time_since_epoch()).count();
}

// First-fit allocator over [0, size) with coalescing frees.
class Pool {
public:
    explicit Pool(size_t size) : size_(size), free_bytes_(size) { free_[0] = size; }
    bool alloc(size_t bytes, size_t& off)
    {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                off = it->first;
                const size_t rest = it->second - bytes;
                free_.erase(it);
                if (rest) free_[off + bytes] = rest;
                free_bytes_ -= bytes;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes)
    {
        free_bytes_ += bytes;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t free_bytes() const { return free_bytes_; }
    size_t size() const { return size_; }

private:
    size_t size_, free_bytes_;
    std::map<size_t, size_t> free_;
};

struct Layout {
    size_t u, v, w, g, ws, total;  // offsets inside the request's block
    size_t ub, wb, wsb;            // bytes of u (= v), w and workspace
};

bool layout_for(tm_kind kind, uint64_t n, Layout& l)
{
    const size_t ws = tm_workspace_bytes(kind, n);
    if (!ws) return false;
    const size_t L = (n + 63) / 64;
    l.ub = L * 8;
    l.wb = (kind == TM_FULL ? 2 * L : L) * 8;
    l.wsb = ws;
    size_t o = 0;
    l.ws = o; o = align_up(o + ws);
    l.u = o; o = align_up(o + l.ub);
    l.v = o; o = align_up(o + l.ub);
    l.w = o; o = align_up(o + l.wb);
    l.g = o; o = align_up(o + sizeof(tm_guard));
    l.total = o;
    return true;
}

struct Job {
    uint64_t id;
    tm_request req;
    tm_guard* guard_host;
    Layout lay;
    size_t off = 0;
    int stream = -1;
    hipEvent_t done = nullptr;
    double t_submit = 0.0;
};

}  // namespace

struct tm_server {
    int dev = 0;
    char* base = nullptr;
    Pool pool;
    std::vector<hipStream_t> streams;
    std::vector<int> load;
    std::vector<hipEvent_t> spare_events;
    std::deque<Job> waiting;
    std::vector<std::deque<Job>> running;  // per stream, in launch order
    size_t n_running = 0;
    std::deque<std::pair<uint64_t, tm_status>> finished;
    uint64_t next_id = 1;
    size_t max_inflight = 0;
    explicit tm_server(size_t bytes) : pool(bytes) {}
};

namespace {

tm_status launch(tm_server* s, Job& j)
{
    hipStream_t st = s->streams[j.stream];
    char* b = s->base + j.off;
    uint64_t* du = reinterpret_cast<uint64_t*>(b + j.lay.u);
    uint64_t* dv = reinterpret_cast<uint64_t*>(b + j.lay.v);
    uint64_t* dw = reinterpret_cast<uint64_t*>(b + j.lay.w);
    tm_guard* dg = reinterpret_cast<tm_guard*>(b + j.lay.g);
    if (hipMemcpyAsync(du, j.req.u, j.lay.ub, hipMemcpyHostToDevice, st) != hipSuccess) return TM_ERR_HIP;
    if (j.req.v == j.req.u) {
        dv = du;  // squaring: one copy
    } else if (hipMemcpyAsync(dv, j.req.v, j.lay.ub, hipMemcpyHostToDevice, st) != hipSuccess) {
        return TM_ERR_HIP;
    }
    tm_status r = tm_mul((tm_kind)j.req.kind, dw, du, dv, j.req.n_bits, b + j.lay.ws, j.lay.wsb, st, dg);
    if (r != TM_OK) return r;
    if (hipMemcpyAsync(j.req.w, dw, j.lay.wb, hipMemcpyDeviceToHost, st) != hipSuccess) return TM_ERR_HIP;
    if (j.guard_host &&
        hipMemcpyAsync(j.guard_host, dg, sizeof(tm_guard), hipMemcpyDeviceToHost, st) != hipSuccess)
        return TM_ERR_HIP;
    if (s->spare_events.empty()) {
        hipEvent_t e;
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return TM_ERR_HIP;
        s->spare_events.push_back(e);
    }
    j.done = s->spare_events.back();
    s->spare_events.pop_back();
    if (hipEventRecord(j.done, st) != hipSuccess) return TM_ERR_HIP;
    return TM_OK;
}

// Admit waiting requests in order while slots and memory allow (see the
// header).
void admit(tm_server* s)
{
    size_t reserved = 0;
    for (auto it = s->waiting.begin(); it != s->waiting.end() && s->n_running < s->max_inflight;) {
        Job& j = *it;
        size_t off;
        const bool room = s->pool.free_bytes() >= reserved + j.lay.total;
        if (room && s->pool.alloc(j.lay.total, off)) {
            j.off = off;
            int best = 0;
            for (int k = 1; k < (int)s->streams.size(); k++)
                if (s->load[k] < s->load[best]) best = k;
            j.stream = best;
            tm_status r = launch(s, j);
            if (r != TM_OK) {
                // the request never reached the device or failed to launch:
                // wait for whatever was queued on its stream, then release
                (void)hipStreamSynchronize(s->streams[best]);
                s->pool.release(j.off, j.lay.total);
                if (j.done) s->spare_events.push_back(j.done);
                s->finished.emplace_back(j.id, r);
            } else {
                s->load[best]++;
                s->running[best].push_back(j);
                s->n_running++;
            }
            it = s->waiting.erase(it);
        } else {
            reserved += j.lay.total;
            ++it;
        }
    }
}

// Work on a stream completes in launch order, so only the oldest request of
// each stream needs an event query (or a wait, when block is set).
void retire(tm_server* s, bool block)
{
    for (auto& q : s->running) {
        while (!q.empty()) {
            Job& j = q.front();
            hipError_t e = block ? hipEventSynchronize(j.done) : hipEventQuery(j.done);
            if (e == hipErrorNotReady) break;
            s->finished.emplace_back(j.id, e == hipSuccess ? TM_OK : TM_ERR_HIP);
            s->pool.release(j.off, j.lay.total);
            s->load[j.stream]--;
            s->spare_events.push_back(j.done);
            q.pop_front();
            s->n_running--;
        }
    }
}

}  // namespace

extern "C" {

size_t tm_server_footprint(tm_kind kind, uint64_t n_bits)
{
    Layout l;
    return layout_for(kind, n_bits, l) ? l.total : 0;
}

tm_status tm_server_create(size_t pool_bytes, int n_streams, int max_inflight, tm_server** out)
{
    if (!out || pool_bytes == 0 || n_streams < 1 || n_streams > 64 || max_inflight < 0)
        return TM_ERR_INVALID;
    *out = nullptr;
    tm_server* s = new (std::nothrow) tm_server(align_up(pool_bytes));
    if (!s) return TM_ERR_INVALID;
    s->max_inflight = max_inflight ? (size_t)max_inflight : (size_t)8 * n_streams;
    if (hipGetDevice(&s->dev) != hipSuccess || hipMalloc(&s->base, s->pool.size()) != hipSuccess) {
        delete s;
        return TM_ERR_HIP;
    }
    for (int k = 0; k < n_streams; k++) {
        hipStream_t st;
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
            tm_server_destroy(s);
            return TM_ERR_HIP;
        }
        s->streams.push_back(st);
        s->load.push_back(0);
        s->running.emplace_back();
    }
    *out = s;
    return TM_OK;
}

tm_status tm_server_submit(tm_server* s, const tm_request* req, tm_guard* guard_host, uint64_t* id)
{
    if (!s || !req || !req->u || !req->v || !req->w || req->kind > 2) return TM_ERR_INVALID;
    Job j;
    if (!layout_for((tm_kind)req->kind, req->n_bits, j.lay)) return TM_ERR_UNSUPPORTED;
    if (j.lay.total > s->pool.size()) return TM_ERR_INVALID;  // can never be admitted
    j.id = s->next_id++;
    j.req = *req;
    j.guard_host = guard_host;
    j.t_submit = now_s();
    if (id) *id = j.id;
    s->waiting.push_back(j);
    admit(s);
    return TM_OK;
}

int tm_server_poll(tm_server* s, uint64_t* ids, tm_status* status, int cap)
{
    if (!s) return -1;
    retire(s, false);
    admit(s);
    int n = 0;
    while (n < cap && !s->finished.empty()) {
        if (ids) ids[n] = s->finished.front().first;
        if (status) status[n] = s->finished.front().second;
        s->finished.pop_front();
        n++;
    }
    return n;
}

size_t tm_server_pending(const tm_server* s)
{
    return s ? s->waiting.size() + s->n_running : 0;
}

tm_status tm_server_drain(tm_server* s)
{
    if (!s) return TM_ERR_INVALID;
    while (!s->waiting.empty() || s->n_running) {
        retire(s, s->waiting.empty());
        admit(s);
    }
    return TM_OK;
}

void tm_server_destroy(tm_server* s)
{
    if (!s) return;
    for (auto& q : s->running)
        for (auto& j : q) (void)hipEventSynchronize(j.done);
    for (auto& q : s->running)
        for (auto& j : q) (void)hipEventDestroy(j.done);
    for (auto e : s->spare_events) (void)hipEventDestroy(e);
    for (auto st : s->streams) (void)hipStreamDestroy(st);
    if (s->base) (void)hipFree(s->base);
    delete s;
}

tm_status tm_serve_trace(const tm_request* reqs, const double* arrival_s, size_t count,
                         size_t pool_bytes, int n_streams, int max_inflight, double* latency_s,
                         tm_guard* guards_host, double* makespan_s)
{
    if ((!reqs || !arrival_s || !latency_s) && count) return TM_ERR_INVALID;
    for (size_t i = 1; i < count; i++)
        if (arrival_s[i] < arrival_s[i - 1]) return TM_ERR_INVALID;
    // build the per-size caches before the clock starts
    {
        hipStream_t st;
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) return TM_ERR_HIP;
        std::map<std::pair<uint32_t, uint64_t>, bool> seen;
        tm_status r = TM_OK;
        for (size_t i = 0; i < count && r == TM_OK; i++) {
            auto key = std::make_pair(reqs[i].kind, reqs[i].n_bits);
            if (seen.count(key)) continue;
            seen[key] = true;
            r = tm_prepare((tm_kind)reqs[i].kind, reqs[i].n_bits, st);
        }
        (void)hipStreamSynchronize(st);
        (void)hipStreamDestroy(st);
        if (r != TM_OK) return r;
    }
    tm_server* s = nullptr;
    tm_status r = tm_server_create(pool_bytes, n_streams, max_inflight, &s);
    if (r != TM_OK) return r;
    std::map<uint64_t, size_t> index;
    std::vector<uint64_t> ids(64);
    std::vector<tm_status> sts(64);
    size_t next = 0, done = 0;
    tm_status first_err = TM_OK;
    const double t0 = now_s();
    while (done < count) {
        const double t = now_s() - t0;
        while (next < count && arrival_s[next] <= t) {
            uint64_t id = 0;
            tm_status q = tm_server_submit(s, &reqs[next], guards_host ? guards_host + next : nullptr, &id);
            if (q != TM_OK) {
                if (first_err == TM_OK) first_err = q;
                latency_s[next] = -1.0;
                done++;
            } else {
                index[id] = next;
            }
            next++;
        }
        const int k = tm_server_poll(s, ids.data(), sts.data(), (int)ids.size());
        if (k < 0) {
            first_err = TM_ERR_INVALID;
            break;
        }
        const double tc = now_s() - t0;
        for (int q = 0; q < k; q++) {
            const size_t i = index[ids[q]];
            index.erase(ids[q]);
            latency_s[i] = sts[q] == TM_OK ? tc - arrival_s[i] : -1.0;
            if (sts[q] != TM_OK && first_err == TM_OK) first_err = sts[q];
            done++;
        }
    }
    if (makespan_s) *makespan_s = now_s() - t0;
    tm_server_destroy(s);
    return first_err;
}

}  // extern "C"
