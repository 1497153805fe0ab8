// Continuous-batching request server.
//
// A request (one array, 1..n frequencies, a scan set) is split into one job per
// frequency.  A fixed set of slots, each a host thread with its own HIP stream
// and persistent device buffers, takes jobs from one FIFO queue: a job is
// admitted as soon as a slot is free and the device bytes that its slot must
// hold for it fit the server's budget, so requests that arrive while others
// run start at once and their kernels overlap on the device.  The per-(array,
// frequency) block spectra come from the context's shared operator cache and
// stay resident across requests; the Krylov workspace of a slot stays
// allocated between jobs.  A job whose slot would have to grow past the budget
// waits at the head of the queue; idle slots then hand their buffers back.
#include <condition_variable>
#include <deque>
#include <thread>
#include <unordered_map>

#include "runtime.h"

namespace {

using namespace mbt;
using Clock = std::chrono::steady_clock;

struct ReqState {
    uint64_t ticket = 0;
    mbt_array arr;
    mbt_solve_opts opts;
    std::vector<double> freq, theta, phi;
    double z0 = 50.0;
    size_t need_ws = 0, need_xs = 0;   // slot bytes for one frequency
    int pending = 0;
    bool started = false, done = false;
    mbt_result* res = nullptr;
};

struct Job {
    std::shared_ptr<ReqState> rq;
    int fi = 0;
};

void free_result(mbt_result* r) {
    if (!r) return;
    delete[] r->Zp;
    delete[] r->Za;
    delete[] r->Gamma;
    delete[] r->Gamma_wave;
    delete[] r->iters_max;
    delete r;
}

}  // namespace

struct mbt_server {
    mbt_ctx* ctx = nullptr;
    size_t budget = 0;
    std::vector<std::unique_ptr<Worker>> slots;
    std::vector<size_t> held;   // bytes each slot holds (kept under mu)
    size_t held_total = 0;
    std::vector<std::thread> threads;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Job> queue;
    std::unordered_map<uint64_t, std::shared_ptr<ReqState>> reqs;
    uint64_t next_ticket = 1;
    bool stopping = false;
    Clock::time_point t0 = Clock::now();

    double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }
    void run_slot(int i);
};

void mbt_server::run_slot(int i) {
    (void)hipSetDevice(ctx->device);
    Worker& w = *slots[i];
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
        if (queue.empty()) {
            if (stopping) break;
            cv_work.wait(lk);
            continue;
        }
        const ReqState& head = *queue.front().rq;
        const size_t want = Worker::grown(w.ws.bytes, head.need_ws) + Worker::grown(w.xs.bytes, head.need_xs);
        const size_t delta = want > held[i] ? want - held[i] : 0;
        if (held_total + delta > budget) {
            if (held[i] > 0) {
                // idle slot: hand the buffers back and look again
                const size_t h = held[i];
                lk.unlock();
                (void)hipStreamSynchronize(w.stream);
                w.ws.release();
                w.xs.release();
                lk.lock();
                held_total -= h;
                held[i] = 0;
                continue;
            }
            cv_work.wait(lk);   // memory frees up when a running job ends
            continue;
        }
        held_total += delta;
        held[i] += delta;
        Job job = queue.front();
        queue.pop_front();
        ReqState& rq = *job.rq;
        if (!rq.started) {
            rq.started = true;
            rq.res->t_start = now();
        }
        lk.unlock();

        int code = MBT_OK;
        int iters = 0;
        try {
            const int P = rq.arr.g.P, ns = (int)rq.theta.size();
            mbt_result* r = rq.res;
            const int64_t zo = (int64_t)job.fi * P * P * 2, so = (int64_t)job.fi * ns * 2;
            mbt_stats st{};
            SolveOut out = solve_frequency(ctx, &rq.arr, rq.freq[job.fi], rq.opts, budget, rq.theta.data(),
                                           rq.phi.data(), ns, rq.z0, r->Zp + zo, ns ? r->Za + so : nullptr,
                                           ns ? r->Gamma + so : nullptr, ns ? r->Gamma_wave + so : nullptr, w, &st);
            code = solve_status(out);
            iters = st.iters_max;
        } catch (const Error& e) {
            code = e.code;
        } catch (const std::bad_alloc&) {
            code = MBT_ENOMEM;
        } catch (const std::exception&) {
            code = MBT_EDEVICE;
        }

        lk.lock();
        // the slot's buffers may have grown inside the job: record what it holds now
        held_total = held_total - held[i] + w.held();
        held[i] = w.held();
        rq.res->iters_max[job.fi] = iters;
        if (code != MBT_OK && rq.res->status == MBT_OK) rq.res->status = (mbt_status)code;
        if (--rq.pending == 0) {
            rq.done = true;
            rq.res->t_done = now();
            cv_done.notify_all();
        }
        cv_work.notify_all();
    }
}

extern "C" {

mbt_status mbt_server_create(mbt_ctx* ctx, int32_t max_inflight, size_t hbm_budget_bytes, mbt_server** out) {
    if (!ctx || !out || max_inflight < 1 || max_inflight > 64) {
        set_last_error("server needs a context, an output handle and 1..64 slots");
        return MBT_EINVAL;
    }
    try {
        MBT_HIP(hipSetDevice(ctx->device));
        std::unique_ptr<mbt_server> s(new mbt_server());
        s->ctx = ctx;
        if (hbm_budget_bytes) {
            s->budget = hbm_budget_bytes;
        } else {
            const size_t reserved = ctx->cache_limit + ctx->main->held();
            s->budget = ctx->budget > reserved ? ctx->budget - reserved : 0;
        }
        if (s->budget == 0) {
            set_last_error("no device memory left for the server");
            return MBT_ENOMEM;
        }
        for (int i = 0; i < max_inflight; ++i) s->slots.emplace_back(new Worker(ctx->device));
        s->held.assign(max_inflight, 0);
        for (int i = 0; i < max_inflight; ++i) s->threads.emplace_back(&mbt_server::run_slot, s.get(), i);
        *out = s.release();
        return MBT_OK;
    } catch (const Error& e) {
        set_last_error(e.what());
        return (mbt_status)e.code;
    } catch (...) {
        set_last_error("device error");
        return MBT_EDEVICE;
    }
}

mbt_status mbt_server_submit(mbt_server* srv, const mbt_request* req, uint64_t* ticket) {
    if (!srv || !req || !ticket) {
        set_last_error("NULL argument");
        return MBT_EINVAL;
    }
    try {
        auto rq = std::make_shared<ReqState>();
        rq->arr.g = make_geom(req->elem, req->lat);
        rq->arr.elem = req->elem;
        rq->arr.lat = req->lat;
        validate_opts(req->opts);
        MBT_REQUIRE(req->nfreq >= 1 && req->nfreq <= 1024 && req->freq_ratio, "nfreq must be in 1..1024");
        MBT_REQUIRE(req->nscan >= 0 && (req->nscan == 0 || (req->theta && req->phi)), "scan arrays missing");
        MBT_REQUIRE(req->z0 > 0 && std::isfinite(req->z0), "z0 must be positive");
        rq->freq.assign(req->freq_ratio, req->freq_ratio + req->nfreq);
        for (double f : rq->freq) MBT_REQUIRE(f > 0 && std::isfinite(f), "freq_ratio must be positive");
        rq->theta.assign(req->theta, req->theta + req->nscan);
        rq->phi.assign(req->phi, req->phi + req->nscan);
        rq->z0 = req->z0;
        rq->opts = req->opts;
        const Geom& g = rq->arr.g;
        // RHS batch: what fits half the budget (two large jobs can overlap), else the whole budget
        rq->need_xs = extract_bytes(g.P, req->nscan);
        const size_t xs_held = Worker::grown(0, rq->need_xs);
        if (xs_held >= srv->budget) throw Error(MBT_ENOMEM, "request does not fit the device-memory budget");
        auto ws_for = [&](int c) {
            return solve_bytes(g, padded(c, rq->opts), rq->opts) + sizeof(int32_t) * (g.P + g.P / c + 1) + 4096;
        };
        int chunk = req->opts.rhs_chunk > 0 ? std::min(req->opts.rhs_chunk, g.P) : g.P;
        if (req->opts.rhs_chunk <= 0) {
            const size_t half = srv->budget / 2;
            while (chunk > 1 && Worker::grown(0, ws_for(chunk)) + xs_held > half) chunk = (chunk + 1) / 2;
            if (Worker::grown(0, ws_for(chunk)) + xs_held > half) chunk = 1;
        }
        rq->need_ws = ws_for(chunk);
        if (Worker::grown(0, rq->need_ws) + xs_held > srv->budget)
            throw Error(MBT_ENOMEM, "request does not fit the device-memory budget");
        rq->opts.rhs_chunk = chunk;
        rq->opts.flags &= ~MBT_FLAG_NO_CACHE;   // served requests share the operator cache

        std::unique_ptr<mbt_result, void (*)(mbt_result*)> r(new mbt_result(), free_result);
        const int nf = req->nfreq, ns = req->nscan;
        const int64_t PP = (int64_t)g.P * g.P;
        r->status = MBT_OK;
        r->nfreq = nf;
        r->nports = g.P;
        r->nscan = ns;
        r->Zp = new double[(size_t)nf * PP * 2]();
        r->Za = new double[(size_t)nf * std::max(ns, 1) * 2]();
        r->Gamma = new double[(size_t)nf * std::max(ns, 1) * 2]();
        r->Gamma_wave = new double[(size_t)nf * std::max(ns, 1) * 2]();
        r->iters_max = new int32_t[nf]();
        std::lock_guard<std::mutex> lk(srv->mu);
        MBT_REQUIRE(!srv->stopping, "server is stopping");
        r->t_submit = srv->now();
        rq->ticket = srv->next_ticket++;
        rq->pending = nf;
        rq->res = r.release();
        srv->reqs[rq->ticket] = rq;
        for (int f = 0; f < nf; ++f) srv->queue.push_back(Job{rq, f});
        *ticket = rq->ticket;
        srv->cv_work.notify_all();
        return MBT_OK;
    } catch (const Error& e) {
        set_last_error(e.what());
        return (mbt_status)e.code;
    } catch (const std::bad_alloc&) {
        set_last_error("host allocation failed");
        return MBT_ENOMEM;
    } catch (...) {
        set_last_error("device error");
        return MBT_EDEVICE;
    }
}

mbt_status mbt_server_wait(mbt_server* srv, uint64_t ticket, int32_t timeout_ms, mbt_result** out) {
    if (!srv || !out) return MBT_EINVAL;
    std::unique_lock<std::mutex> lk(srv->mu);
    auto it = srv->reqs.find(ticket);
    if (it == srv->reqs.end()) {
        set_last_error("unknown ticket");
        return MBT_EINVAL;
    }
    std::shared_ptr<ReqState> rq = it->second;
    if (timeout_ms < 0) {
        srv->cv_done.wait(lk, [&] { return rq->done; });
    } else if (!srv->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), [&] { return rq->done; })) {
        set_last_error("request not finished within the timeout");
        return MBT_ETIMEOUT;
    }
    *out = rq->res;
    rq->res = nullptr;
    srv->reqs.erase(ticket);
    return MBT_OK;
}

void mbt_result_free(mbt_result* res) { free_result(res); }

double mbt_server_clock(const mbt_server* srv) { return srv ? srv->now() : 0.0; }

void mbt_server_destroy(mbt_server* srv) {
    if (!srv) return;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stopping = true;
        srv->cv_work.notify_all();
    }
    for (auto& t : srv->threads) t.join();
    for (auto& kv : srv->reqs) free_result(kv.second->res);
    (void)hipSetDevice(srv->ctx->device);
    srv->slots.clear();
    delete srv;
}

}  // extern "C"
