// Request server (mcmf_server_*): resident graphs, admission by a device
// memory budget, continuous batching over several streams.
//
// Threads: one dispatcher and one worker per stream slot.  The dispatcher
// forms a batch from the arrival queue whenever a slot is idle: requests join
// while the batch's admission estimate fits the budget left by the batches
// in flight (arrival order is kept; a request larger than the whole budget
// runs alone once nothing else is in flight).  A request above
// max_batch_steps runs alone, and while max_large_in_flight such requests
// run, further large ones wait while the requests behind them go ahead.  The slot's
// worker runs the batch with mcmf_batch on its own stream, then releases
// the estimate and completes the tickets.  If a batch fails as a whole, its
// requests are run again one at a time so that one failure stays with its
// own request.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "ops.hpp"

namespace mcmf {

namespace {

using Clock = std::chrono::steady_clock;

double ms_between(Clock::time_point a, Clock::time_point b) {
    return std::chrono::duration<double, std::milli>(b - a).count();
}

struct Ticket {
    uint64_t id = 0;
    mcmf_request *req = nullptr;
    uint64_t fixed_bytes = 0;  // per-request arrays
    uint64_t visit_bytes = 0;  // upper bound of its visit records
    uint64_t steps = 0;        // upper bound of its walk steps
    Clock::time_point submitted, started, finished;
    int32_t batch_size = 0;
    bool done = false;
    std::string error; // the failing call's message (the slot thread's last error)
};

// Host-side sizing of one request, from sizes alone (no device access, so
// submitting never waits behind the batches in flight):
//  * device bytes it holds while its batch runs, without the shared
//    visit-record buffer (an upper bound);
//  * its visit-record bytes and walk steps (estimates: a diagonal request on
//    a row subset starts walks from the neighbours of its rows, taken as
//    count * mean row length, at most every row with entries).
void estimate(const mcmf_request &q, uint64_t *fixed, uint64_t *visits, uint64_t *steps) {
    const mcmf_graph *g = q.graph;
    const uint64_t n = static_cast<uint64_t>(g->n);
    const uint64_t kb = q.K >= 2 ? static_cast<uint64_t>(q.K) : 2;
    uint64_t f = 8 * kb + 64 * 1024; // coefficients, descriptors, rounding slack
    uint64_t starts = q.K >= 2 ? static_cast<uint64_t>(g->n_active) : 0;
    if (q.kind == MCMF_REQ_ACTION) {
        f += 8 * n * 4; // v and out staging, r, q
        // Value records when the graph's tuning uses them (an upper bound:
        // a batch may fall back to EDGE walks when they do not fit).
        if (q.K >= 2 && g->tuning.action_sampler == MCMF_SAMPLER_VALUE && !g->weighted && !q.path_digest)
            f += 16 * static_cast<uint64_t>(g->nnz);
    } else {
        const uint64_t count = q.rows ? static_cast<uint64_t>(q.n_rows) : n;
        f += 8 * n + 2 * n + 4 * n + 8 * (n + 1) + 12 * count; // dacc, marks, start list, items, rows/out
        if (q.rows && n > 0) {
            const uint64_t mean_len = (static_cast<uint64_t>(g->nnz) + n - 1) / n;
            starts = std::min(starts, count * std::max<uint64_t>(mean_len, 1));
        }
    }
    if (q.path_digest)
        f += 8 * n;
    const uint64_t per = q.precision == MCMF_PRECISION_FP32_WEIGHTS ? 8 : 12;
    const uint64_t st = q.K >= 2 ? starts * static_cast<uint64_t>(q.n_walks) * (kb - 1) : 0;
    *fixed = f;
    *visits = q.kind == MCMF_REQ_DIAG ? st * per : 0;
    *steps = st;
}

} // namespace

} // namespace mcmf

struct mcmf_server {
    mcmf_server_opts opts = {};
    std::mutex mu;
    std::condition_variable cv_dispatch; // queue, slot or memory changed
    std::condition_variable cv_done;     // a ticket completed
    std::deque<std::shared_ptr<mcmf::Ticket>> queue;
    std::unordered_map<uint64_t, std::shared_ptr<mcmf::Ticket>> tickets;
    uint64_t next_id = 1;
    bool stopping = false;
    bool dispatch_done = false; // the dispatcher has handed out the last batch
    uint64_t in_flight = 0;
    mcmf_server_stats stats = {};
    uint64_t batches_in_flight = 0;
    int32_t large_in_flight = 0;

    struct Slot {
        hipStream_t stream = nullptr;
        std::thread worker;
        std::vector<std::shared_ptr<mcmf::Ticket>> batch;
        uint64_t est = 0;
        bool busy = false;
        bool large = false; // its batch is one request above max_batch_steps
    };
    std::vector<std::unique_ptr<Slot>> slots;
    std::condition_variable cv_slot; // a slot received a batch
    std::thread dispatcher;
};

namespace mcmf {

namespace {

uint64_t batch_steps(const std::vector<std::shared_ptr<Ticket>> &b) {
    uint64_t steps = 0;
    for (const auto &t : b)
        steps += t->steps;
    return steps;
}

uint64_t batch_estimate(const std::vector<std::shared_ptr<Ticket>> &b, uint64_t chunk) {
    uint64_t fixed = 0, visits = 0;
    for (const auto &t : b) {
        fixed += t->fixed_bytes;
        visits += t->visit_bytes;
    }
    return fixed + std::min(visits, chunk);
}

void run_slot(mcmf_server *S, mcmf_server::Slot *slot) {
    (void)hipSetDevice(S->opts.device);
    // This thread's allocations and copies must not invalidate another slot's
    // hipGraph capture (the default, global interaction mode would).
    hipStreamCaptureMode mode = hipStreamCaptureModeRelaxed;
    (void)hipThreadExchangeStreamCaptureMode(&mode);
    for (;;) {
        std::vector<std::shared_ptr<Ticket>> batch;
        {
            std::unique_lock<std::mutex> lock(S->mu);
            // Exit only once the dispatcher is done: until then a stopping
            // server still hands queued requests to idle slots.
            S->cv_slot.wait(lock, [&] { return !slot->batch.empty() || S->dispatch_done; });
            if (slot->batch.empty())
                return;
            batch = slot->batch;
        }
        const Clock::time_point t0 = Clock::now();
        std::vector<mcmf_request> reqs(batch.size());
        for (size_t i = 0; i < batch.size(); ++i)
            reqs[i] = *batch[i]->req;
        mcmf_batch_opts bo = {};
        bo.stream = slot->stream;
        bo.use_graph = S->opts.use_graph;
        bo.visit_chunk_bytes = S->opts.visit_chunk_bytes;
        std::vector<std::string> errors(reqs.size());
        Status st = run_batch(reqs.data(), static_cast<int64_t>(reqs.size()), &bo, nullptr);
        if (st && reqs.size() > 1) {
            // Isolate the failure: every request on its own.
            for (size_t i = 0; i < reqs.size(); ++i) {
                mcmf_request one = reqs[i];
                Status s1 = run_batch(&one, 1, &bo, nullptr);
                reqs[i].status = s1.code;
                reqs[i].walk_steps = s1 ? 0 : one.walk_steps;
                if (s1)
                    errors[i] = mcmf_last_error();
            }
        } else if (st) {
            reqs[0].status = st.code;
            errors[0] = mcmf_last_error();
        }
        const Clock::time_point t1 = Clock::now();
        {
            std::lock_guard<std::mutex> lock(S->mu);
            for (size_t i = 0; i < batch.size(); ++i) {
                Ticket &t = *batch[i];
                t.req->status = reqs[i].status;
                t.req->walk_steps = reqs[i].walk_steps;
                t.started = t0;
                t.finished = t1;
                t.batch_size = static_cast<int32_t>(batch.size());
                t.error = errors[i];
                t.done = true;
            }
            S->in_flight -= slot->est;
            S->stats.completed += batch.size();
            S->stats.bytes_in_flight = S->in_flight;
            --S->batches_in_flight;
            if (slot->large)
                --S->large_in_flight;
            slot->batch.clear();
            slot->est = 0;
            slot->busy = false;
            slot->large = false;
        }
        S->cv_done.notify_all();
        S->cv_dispatch.notify_all();
    }
}

void run_dispatcher(mcmf_server *S) {
    const uint64_t budget = S->opts.hbm_budget_bytes;
    const uint64_t chunk = S->opts.visit_chunk_bytes;
    std::unique_lock<std::mutex> lock(S->mu);
    for (;;) {
        mcmf_server::Slot *free_slot = nullptr;
        for (auto &sl : S->slots)
            if (!sl->busy) {
                free_slot = sl.get();
                break;
            }
        if (S->queue.empty() || !free_slot) {
            if (S->stopping && S->queue.empty())
                break;
            S->cv_dispatch.wait(lock);
            continue;
        }
        // Form a batch from the queue in arrival order.  A large request (above
        // max_batch_steps: it runs alone) while max_large_in_flight of them
        // already run is passed over, and so is everything when the head does
        // not fit the memory budget; smaller requests behind a passed-over
        // large one may go first.
        std::vector<std::shared_ptr<Ticket>> batch;
        uint64_t est = 0;
        bool large = false;
        for (auto it = S->queue.begin(); it != S->queue.end() &&
                                         static_cast<int32_t>(batch.size()) < S->opts.max_batch;) {
            const bool big = (*it)->steps > S->opts.max_batch_steps;
            if (big && (!batch.empty() || S->large_in_flight >= S->opts.max_large_in_flight)) {
                if (!batch.empty())
                    break; // a large request ends the batch (it runs alone)
                ++it;
                continue;
            }
            batch.push_back(*it);
            const uint64_t e = batch_estimate(batch, chunk);
            const bool fits = budget == 0 || S->in_flight + e <= budget;
            const bool alone = batch.size() == 1 && S->in_flight == 0;
            // A batch completes as a unit: later requests join only while the
            // batch stays small, so small requests do not wait for a large one.
            const bool small = batch.size() == 1 || batch_steps(batch) <= S->opts.max_batch_steps;
            if ((!fits && !alone) || !small) {
                batch.pop_back();
                break;
            }
            est = e;
            it = S->queue.erase(it);
            if (big) {
                large = true;
                break;
            }
        }
        if (batch.empty()) {
            // Nothing can start next to the batches in flight: wait for one to end.
            S->cv_dispatch.wait(lock);
            continue;
        }
        if (large) {
            ++S->large_in_flight;
            S->stats.peak_large_in_flight =
                std::max<uint64_t>(S->stats.peak_large_in_flight, static_cast<uint64_t>(S->large_in_flight));
        }
        S->in_flight += est;
        ++S->batches_in_flight;
        ++S->stats.batches;
        S->stats.bytes_in_flight = S->in_flight;
        S->stats.peak_bytes_in_flight = std::max(S->stats.peak_bytes_in_flight, S->in_flight);
        S->stats.peak_batches_in_flight = std::max(S->stats.peak_batches_in_flight, S->batches_in_flight);
        S->stats.largest_batch = std::max<uint64_t>(S->stats.largest_batch, batch.size());
        free_slot->batch = std::move(batch);
        free_slot->est = est;
        free_slot->busy = true;
        free_slot->large = large;
        S->cv_slot.notify_all();
    }
    // Wake the workers so that they see the stop.
    S->dispatch_done = true;
    lock.unlock();
    S->cv_slot.notify_all();
}

void stop_server(mcmf_server *S) {
    {
        std::lock_guard<std::mutex> lock(S->mu);
        S->stopping = true;
    }
    S->cv_dispatch.notify_all();
    if (S->dispatcher.joinable())
        S->dispatcher.join();
    S->cv_slot.notify_all();
    for (auto &sl : S->slots)
        if (sl->worker.joinable())
            sl->worker.join();
    for (auto &sl : S->slots)
        if (sl->stream)
            (void)hipStreamDestroy(sl->stream);
}

Status create_server(const mcmf_server_opts *o, mcmf_server **out) {
    if (!out)
        return fail(MCMF_E_ARG, "out is NULL");
    *out = nullptr;
    mcmf_server_opts op = {};
    if (o)
        op = *o;
    for (uint32_t r : op.reserved)
        if (r)
            return fail(MCMF_E_ARG, "reserved option words must be zero");
    if (op.n_streams == 0)
        op.n_streams = 2;
    if (op.max_batch == 0)
        op.max_batch = 64;
    if (op.visit_chunk_bytes == 0)
        op.visit_chunk_bytes = uint64_t(256) << 20;
    if (op.max_batch_steps == 0)
        op.max_batch_steps = uint64_t(1) << 28;
    if (op.max_large_in_flight == 0)
        op.max_large_in_flight = 1;
    if (op.n_streams < 1 || op.n_streams > 16)
        return fail(MCMF_E_ARG, "n_streams = %d outside 1..16", op.n_streams);
    if (op.max_large_in_flight < 1 || op.max_large_in_flight > op.n_streams)
        return fail(MCMF_E_ARG, "max_large_in_flight = %d outside 1..n_streams", op.max_large_in_flight);
    if (op.max_batch < 1)
        return fail(MCMF_E_ARG, "max_batch = %d is below 1", op.max_batch);
    if (op.use_graph != 0 && op.use_graph != 1)
        return fail(MCMF_E_ARG, "use_graph must be 0 or 1");
    int n_dev = 0;
    MCMF_HIP(hipGetDeviceCount(&n_dev));
    if (op.device < 0 || op.device >= n_dev)
        return fail(MCMF_E_ARG, "device %d outside [0, %d)", op.device, n_dev);
    MCMF_HIP(hipSetDevice(op.device));
    std::unique_ptr<mcmf_server> S(new mcmf_server());
    S->opts = op;
    for (int i = 0; i < op.n_streams; ++i) {
        std::unique_ptr<mcmf_server::Slot> sl(new mcmf_server::Slot());
        hipError_t e = hipStreamCreateWithFlags(&sl->stream, hipStreamNonBlocking);
        if (e != hipSuccess) {
            for (auto &x : S->slots)
                (void)hipStreamDestroy(x->stream);
            return hip_fail(e, "hipStreamCreateWithFlags", __FILE__, __LINE__);
        }
        S->slots.push_back(std::move(sl));
    }
    mcmf_server *raw = S.get();
    for (auto &sl : S->slots)
        sl->worker = std::thread(run_slot, raw, sl.get());
    S->dispatcher = std::thread(run_dispatcher, raw);
    *out = S.release();
    return {};
}

Status submit(mcmf_server *S, mcmf_request *req, uint64_t *ticket) {
    if (!S || !req || !ticket)
        return fail(MCMF_E_ARG, "server, request and ticket must not be NULL");
    *ticket = 0;
    mcmf_request copy = *req;
    Status st = check_request(copy);
    if (st) {
        req->status = st.code;
        return st;
    }
    if (copy.graph->device != S->opts.device)
        return fail(MCMF_E_ARG, "the request's graph lives on device %d, the server on %d",
                    copy.graph->device, S->opts.device);
    auto t = std::make_shared<Ticket>();
    t->req = req;
    estimate(copy, &t->fixed_bytes, &t->visit_bytes, &t->steps);
    t->submitted = Clock::now();
    {
        std::lock_guard<std::mutex> lock(S->mu);
        if (S->stopping)
            return fail(MCMF_E_ARG, "the server is stopping");
        t->id = S->next_id++;
        S->tickets[t->id] = t;
        S->queue.push_back(t);
        ++S->stats.submitted;
        *ticket = t->id;
    }
    S->cv_dispatch.notify_all();
    return {};
}

Status wait_ticket(mcmf_server *S, uint64_t id, mcmf_ticket_info *info) {
    if (!S)
        return fail(MCMF_E_ARG, "server is NULL");
    std::shared_ptr<Ticket> t;
    {
        std::unique_lock<std::mutex> lock(S->mu);
        auto it = S->tickets.find(id);
        if (it == S->tickets.end())
            return fail(MCMF_E_ARG, "unknown ticket %llu", static_cast<unsigned long long>(id));
        t = it->second;
        S->cv_done.wait(lock, [&] { return t->done; });
        S->tickets.erase(id);
    }
    const mcmf_status code = t->req->status;
    if (info) {
        memset(info, 0, sizeof *info);
        info->status = code;
        info->batch_size = t->batch_size;
        info->queue_ms = ms_between(t->submitted, t->started);
        info->run_ms = ms_between(t->started, t->finished);
        info->est_bytes = t->fixed_bytes + std::min(t->visit_bytes, S->opts.visit_chunk_bytes);
        info->est_steps = t->steps;
    }
    if (code != MCMF_OK)
        return fail(code, "request failed: %s", t->error.empty() ? mcmf_status_string(code) : t->error.c_str());
    return {};
}

} // namespace

} // namespace mcmf

extern "C" mcmf_status mcmf_server_create(const mcmf_server_opts *opts, mcmf_server **out) {
    mcmf::clear_error();
    return mcmf::create_server(opts, out).code;
}

extern "C" mcmf_status mcmf_server_submit(mcmf_server *s, mcmf_request *req, uint64_t *ticket) {
    mcmf::clear_error();
    return mcmf::submit(s, req, ticket).code;
}

extern "C" mcmf_status mcmf_server_wait(mcmf_server *s, uint64_t ticket, mcmf_ticket_info *info) {
    mcmf::clear_error();
    return mcmf::wait_ticket(s, ticket, info).code;
}

extern "C" mcmf_status mcmf_server_query(mcmf_server *s, mcmf_server_stats *stats) {
    mcmf::clear_error();
    if (!s || !stats) {
        mcmf::fail(MCMF_E_ARG, "server and stats must not be NULL");
        return MCMF_E_ARG;
    }
    std::lock_guard<std::mutex> lock(s->mu);
    *stats = s->stats;
    return MCMF_OK;
}

extern "C" void mcmf_server_destroy(mcmf_server *s) {
    if (!s)
        return;
    mcmf::stop_server(s);
    delete s;
}
