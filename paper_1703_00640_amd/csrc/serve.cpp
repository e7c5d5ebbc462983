// Continuous-batching server of the truncated-multiplication library (see
// the tm_server_* declarations in include/tmul.h).
//
// A server owns one device memory pool and a few HIP streams.  Requests
// carry host operand / result buffers and wait in arrival order.  Whenever
// a stream has room for another batch, the waiting requests whose device
// footprint (operands, result, workspace) can be carved out of the pool are
// admitted together, up to kMaxBatch, and run as one batch on that stream:
// operands in, one packed multiplication call (every stage one launch per
// kernel instance), results and guards out, one completion event.  Polling
// retires finished batches, returns their memory and admits more, so
// requests that arrive while others run gather into the next batch, and
// batches on different streams overlap on the device.  A request that does
// not fit reserves the bytes it is waiting for, so smaller requests behind
// it can pass it only within the remaining space (no starvation of large
// requests).
#include <hip/hip_runtime.h>

#include <algorithm>
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

// A request's own pool block holds its workspace and operands; its result
// goes to its batch's result region, where the results of a batch are
// contiguous (so results bound for contiguous host memory leave in one copy).
struct Layout {
    size_t u, v, ws, total;  // offsets inside the request's block, block bytes
    size_t ub, wb, wsb;      // bytes of u (= v), w and workspace
    size_t footprint;        // block + result bytes (tm_server_footprint)
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
    l.total = o;
    l.footprint = o + align_up(l.wb);
    return true;
}

struct Job {
    uint64_t id;
    tm_request req;
    tm_guard* guard_host;
    Layout lay;
    size_t off = 0;
    double t_submit = 0.0;
};

// Requests launched together: one packed multiplication call, one metadata
// and guard block in the pool, one completion event.
struct Batch {
    std::vector<Job> jobs;
    int stream = -1;
    size_t meta_off = 0;
    size_t res_off = 0, res_bytes = 0;  // result region: the jobs' results in order
    hipEvent_t done = nullptr;
    tm_guard* guards_host = nullptr;  // pinned staging of the batch's guards
    char* meta_host = nullptr;        // pinned staging of its launch metadata (graph mode)
    hipGraphExec_t graph = nullptr;   // the batch as one captured graph (graph mode)
};

constexpr size_t kMaxBatch = 64;
// Smallest batch captured as a graph in the automatic graph mode: one graph
// launch replaces about one kernel launch per request and stage plus the
// copies, which pays once the batch is large enough to outweigh the
// capture and instantiation.
constexpr size_t kGraphMinBatch = 16;

// Pool block of a batch: launch metadata, then the guards of its requests.
size_t batch_guard_offset() { return align_up(tm_batch_meta_bytes(kMaxBatch)); }
size_t batch_block_bytes() { return batch_guard_offset() + align_up(kMaxBatch * sizeof(tm_guard)); }

}  // namespace

struct tm_server {
    int dev = 0;
    char* base = nullptr;
    Pool pool;
    std::vector<hipStream_t> streams;
    std::vector<int> load;                 // requests in flight per stream
    std::vector<hipEvent_t> spare_events;
    std::vector<tm_guard*> spare_guards;   // pinned guard staging buffers
    std::vector<char*> spare_meta;         // pinned metadata staging buffers (graph mode)
    int graphs = 0;                        // batches as captured HIP graphs: 0 never,
                                           // 1 every batch of 2 or more, 2 batches of
                                           // kGraphMinBatch or more
    std::deque<Job> waiting;
    std::vector<std::deque<Batch>> running;  // per stream, in launch order
    size_t n_running = 0;
    std::deque<std::pair<uint64_t, tm_status>> finished;
    uint64_t next_id = 1;
    size_t max_inflight = 0;
    explicit tm_server(size_t bytes) : pool(bytes) {}
};

namespace {

// Enqueue a batch's copies, multiplication and guard copy on stream st.
tm_status enqueue(tm_server* s, Batch& b, hipStream_t st)
{
    const size_t k = b.jobs.size();
    char* meta = s->base + b.meta_off;
    tm_guard* dg = reinterpret_cast<tm_guard*>(meta + batch_guard_offset());
    std::vector<tm_request> reqs(k);
    std::vector<void*> wss(k);
    std::vector<size_t> wsb(k);
    std::vector<tm_guard*> gs(k);
    size_t wpos = 0;
    for (size_t i = 0; i < k; i++) {
        Job& j = b.jobs[i];
        char* blk = s->base + j.off;
        uint64_t* du = reinterpret_cast<uint64_t*>(blk + j.lay.u);
        uint64_t* dv = reinterpret_cast<uint64_t*>(blk + j.lay.v);
        if (hipMemcpyAsync(du, j.req.u, j.lay.ub, hipMemcpyHostToDevice, st) != hipSuccess) return TM_ERR_HIP;
        if (j.req.v == j.req.u) {
            dv = du;  // squaring: one copy
        } else if (hipMemcpyAsync(dv, j.req.v, j.lay.ub, hipMemcpyHostToDevice, st) != hipSuccess) {
            return TM_ERR_HIP;
        }
        reqs[i] = j.req;
        reqs[i].u = du;
        reqs[i].v = dv;
        reqs[i].w = reinterpret_cast<uint64_t*>(s->base + b.res_off) + wpos;
        wpos += j.lay.wb / 8;
        wss[i] = blk + j.lay.ws;
        wsb[i] = j.lay.wsb;
        gs[i] = dg + i;
    }
    tm_status r;
    if (k == 1)
        r = tm_mul((tm_kind)reqs[0].kind, reqs[0].w, reqs[0].u, reqs[0].v, reqs[0].n_bits, wss[0],
                   b.jobs[0].lay.wsb, st, gs[0]);
    else if (b.meta_host)
        r = tm_mul_packed_staged(reqs.data(), k, wss.data(), wsb.data(), meta, batch_guard_offset(),
                                 b.meta_host, tm_batch_meta_bytes(kMaxBatch), st, gs.data());
    else
        r = tm_mul_packed(reqs.data(), k, wss.data(), wsb.data(), meta, batch_guard_offset(), st, gs.data());
    if (r != TM_OK) return r;
    // results: one copy per run of requests whose host buffers follow each
    // other (the device results of a batch are contiguous)
    for (size_t i = 0; i < k;) {
        size_t bytes = b.jobs[i].lay.wb, e = i + 1;
        while (e < k && reinterpret_cast<char*>(b.jobs[e - 1].req.w) + b.jobs[e - 1].lay.wb ==
                            reinterpret_cast<char*>(b.jobs[e].req.w)) {
            bytes += b.jobs[e].lay.wb;
            e++;
        }
        if (hipMemcpyAsync(b.jobs[i].req.w, reqs[i].w, bytes, hipMemcpyDeviceToHost, st) != hipSuccess)
            return TM_ERR_HIP;
        i = e;
    }
    if (hipMemcpyAsync(b.guards_host, dg, k * sizeof(tm_guard), hipMemcpyDeviceToHost, st) != hipSuccess)
        return TM_ERR_HIP;
    return TM_OK;
}

// Launch a batch: directly on its stream, or (graph mode) captured into a
// HIP graph that is instantiated and launched as one unit.  A batch whose
// capture fails (for instance pageable host buffers) is launched directly.
tm_status launch(tm_server* s, Batch& b)
{
    hipStream_t st = s->streams[b.stream];
    // host staging buffers are taken before any capture begins
    if (s->spare_guards.empty()) {
        void* h = nullptr;
        if (hipHostMalloc(&h, kMaxBatch * sizeof(tm_guard), hipHostMallocDefault) != hipSuccess) return TM_ERR_HIP;
        s->spare_guards.push_back(static_cast<tm_guard*>(h));
    }
    b.guards_host = s->spare_guards.back();
    s->spare_guards.pop_back();
    const size_t gmin = s->graphs == 1 ? 2 : s->graphs == 2 ? kGraphMinBatch : SIZE_MAX;
    if (b.jobs.size() >= gmin) {
        if (s->spare_meta.empty()) {
            void* h = nullptr;
            if (hipHostMalloc(&h, tm_batch_meta_bytes(kMaxBatch), hipHostMallocDefault) != hipSuccess)
                return TM_ERR_HIP;
            s->spare_meta.push_back(static_cast<char*>(h));
        }
        b.meta_host = s->spare_meta.back();
        s->spare_meta.pop_back();
        hipGraph_t g = nullptr;
        bool ok = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) == hipSuccess;
        if (ok) {
            const tm_status r = enqueue(s, b, st);
            ok = hipStreamEndCapture(st, &g) == hipSuccess && r == TM_OK && g;
        }
        if (ok) ok = hipGraphInstantiate(&b.graph, g, nullptr, nullptr, 0) == hipSuccess;
        if (g) (void)hipGraphDestroy(g);
        if (ok) {
            if (hipGraphLaunch(b.graph, st) != hipSuccess) return TM_ERR_HIP;
        } else {
            if (b.graph) (void)hipGraphExecDestroy(b.graph);
            b.graph = nullptr;
            (void)hipGetLastError();
            const tm_status r = enqueue(s, b, st);
            if (r != TM_OK) return r;
        }
    } else {
        const tm_status r = enqueue(s, b, st);
        if (r != TM_OK) return r;
    }
    if (s->spare_events.empty()) {
        hipEvent_t e;
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return TM_ERR_HIP;
        s->spare_events.push_back(e);
    }
    b.done = s->spare_events.back();
    s->spare_events.pop_back();
    if (hipEventRecord(b.done, st) != hipSuccess) return TM_ERR_HIP;
    return TM_OK;
}

void release_batch(tm_server* s, Batch& b)
{
    for (auto& j : b.jobs) s->pool.release(j.off, j.lay.total);
    if (b.res_bytes) s->pool.release(b.res_off, b.res_bytes);
    s->pool.release(b.meta_off, batch_block_bytes());
    if (b.done) s->spare_events.push_back(b.done);
    if (b.guards_host) s->spare_guards.push_back(b.guards_host);
    if (b.meta_host) s->spare_meta.push_back(b.meta_host);
    if (b.graph) (void)hipGraphExecDestroy(b.graph);
    b.done = nullptr;
    b.guards_host = nullptr;
    b.meta_host = nullptr;
    b.graph = nullptr;
}

// Batches in flight per stream: one running and one queued behind it, so
// requests that arrive meanwhile gather into the next batch.
constexpr size_t kBatchesPerStream = 2;

// The stream with the fewest batches in flight, or -1 if all are full.
int free_stream(const tm_server* s)
{
    int best = -1;
    for (int k = 0; k < (int)s->streams.size(); k++) {
        if (s->running[k].size() >= kBatchesPerStream) continue;
        if (best < 0 || s->running[k].size() < s->running[best].size() ||
            (s->running[k].size() == s->running[best].size() && s->load[k] < s->load[best]))
            best = k;
    }
    return best;
}

void start(tm_server* s, Batch& b)
{
    tm_status r = launch(s, b);
    if (r != TM_OK) {
        // the batch never reached the device or failed to launch: wait for
        // whatever was queued on its stream, then release
        (void)hipStreamSynchronize(s->streams[b.stream]);
        for (auto& j : b.jobs) s->finished.emplace_back(j.id, r);
        release_batch(s, b);
        return;
    }
    s->load[b.stream] += (int)b.jobs.size();
    s->n_running += b.jobs.size();
    s->running[b.stream].push_back(std::move(b));
}

// Admit waiting requests in order while a stream has room for a batch and
// memory allows (see the header), up to kMaxBatch requests per batch.
void admit(tm_server* s)
{
    size_t reserved = 0;
    auto it = s->waiting.begin();
    while (it != s->waiting.end() && s->n_running < s->max_inflight) {
        const int st = free_stream(s);
        if (st < 0) break;
        Batch cur;
        cur.stream = st;
        if (s->pool.free_bytes() < reserved + batch_block_bytes() ||
            !s->pool.alloc(batch_block_bytes(), cur.meta_off))
            break;
        while (it != s->waiting.end() && cur.jobs.size() < kMaxBatch &&
               s->n_running + cur.jobs.size() < s->max_inflight) {
            Job& j = *it;
            size_t off;
            const bool room = s->pool.free_bytes() >= reserved + j.lay.footprint;
            if (room && s->pool.alloc(j.lay.total, off)) {
                j.off = off;
                cur.jobs.push_back(j);
                it = s->waiting.erase(it);
            } else {
                reserved += j.lay.footprint;
                ++it;
            }
        }
        // the batch's result region: if it does not fit, requests go back
        // to the queue (in submission order) from the end of the batch
        bool shrunk = false;
        while (!cur.jobs.empty()) {
            size_t rb = 0;
            for (const Job& j : cur.jobs) rb += j.lay.wb;
            rb = align_up(rb);
            if (s->pool.alloc(rb, cur.res_off)) {
                cur.res_bytes = rb;
                break;
            }
            const Job j = cur.jobs.back();
            cur.jobs.pop_back();
            s->pool.release(j.off, j.lay.total);
            auto pos = std::upper_bound(s->waiting.begin(), s->waiting.end(), j.id,
                                        [](uint64_t id, const Job& w) { return id < w.id; });
            s->waiting.insert(pos, j);
            shrunk = true;
        }
        if (cur.jobs.empty()) {
            s->pool.release(cur.meta_off, batch_block_bytes());
            break;
        }
        start(s, cur);
        if (shrunk) break;  // the queue changed under the iterator
    }
}

// Work on a stream completes in launch order, so only the oldest batch of
// each stream needs an event query (or a wait, when block is set).
void retire(tm_server* s, bool block)
{
    for (auto& q : s->running) {
        while (!q.empty()) {
            Batch& b = q.front();
            hipError_t e = block ? hipEventSynchronize(b.done) : hipEventQuery(b.done);
            if (e == hipErrorNotReady) break;
            for (size_t i = 0; i < b.jobs.size(); i++) {
                const Job& j = b.jobs[i];
                if (j.guard_host && e == hipSuccess) memcpy(j.guard_host, b.guards_host + i, sizeof(tm_guard));
                s->finished.emplace_back(j.id, e == hipSuccess ? TM_OK : TM_ERR_HIP);
            }
            s->load[b.stream] -= (int)b.jobs.size();
            s->n_running -= b.jobs.size();
            release_batch(s, b);
            q.pop_front();
        }
    }
}

}  // namespace

extern "C" {

size_t tm_server_footprint(tm_kind kind, uint64_t n_bits)
{
    Layout l;
    return layout_for(kind, n_bits, l) ? l.footprint : 0;
}

tm_status tm_server_create(size_t pool_bytes, int n_streams, int max_inflight, tm_server** out)
{
    if (!out || pool_bytes == 0 || n_streams < 1 || n_streams > 64 || max_inflight < 0)
        return TM_ERR_INVALID;
    *out = nullptr;
    tm_server* s = new (std::nothrow) tm_server(align_up(pool_bytes));
    if (!s) return TM_ERR_INVALID;
    s->max_inflight = max_inflight ? (size_t)max_inflight : kMaxBatch * kBatchesPerStream * n_streams;
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
    if (j.lay.footprint + batch_block_bytes() > s->pool.size()) return TM_ERR_INVALID;  // can never be admitted
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
        for (auto& b : q) (void)hipEventSynchronize(b.done);
    for (auto& q : s->running)
        for (auto& b : q) {
            (void)hipEventDestroy(b.done);
            (void)hipHostFree(b.guards_host);
            if (b.meta_host) (void)hipHostFree(b.meta_host);
            if (b.graph) (void)hipGraphExecDestroy(b.graph);
        }
    for (auto e : s->spare_events) (void)hipEventDestroy(e);
    for (auto g : s->spare_guards) (void)hipHostFree(g);
    for (auto m : s->spare_meta) (void)hipHostFree(m);
    for (auto st : s->streams) (void)hipStreamDestroy(st);
    if (s->base) (void)hipFree(s->base);
    delete s;
}

tm_status tm_server_use_graphs(tm_server* s, int mode)
{
    if (!s || mode < 0 || mode > 2) return TM_ERR_INVALID;
    s->graphs = mode;
    return TM_OK;
}

tm_status tm_serve_trace(const tm_request* reqs, const double* arrival_s, size_t count,
                         size_t pool_bytes, int n_streams, int max_inflight, double* latency_s,
                         tm_guard* guards_host, double* makespan_s)
{
    return tm_serve_trace_ex(reqs, arrival_s, count, pool_bytes, n_streams, max_inflight, latency_s,
                             guards_host, makespan_s, 0);
}

tm_status tm_serve_trace_ex(const tm_request* reqs, const double* arrival_s, size_t count,
                            size_t pool_bytes, int n_streams, int max_inflight, double* latency_s,
                            tm_guard* guards_host, double* makespan_s, int flags)
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
    s->graphs = (flags & TM_SERVE_GRAPHS_AUTO) ? 2 : (flags & TM_SERVE_GRAPHS) ? 1 : 0;
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
