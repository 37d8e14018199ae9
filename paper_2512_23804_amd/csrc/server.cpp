// Continuous-batching solve server.
//
// Requests (steady problems) are queued by sg_submit.  A scheduler thread
// admits queued requests in arrival order while their estimated device
// footprint fits the HBM budget and a slot is free, groups admitted requests
// of the same shape (n, M, P, precision, solver options) into one batch, and
// hands each batch to a worker thread that owns its own HIP stream.  Batches
// on different workers overlap on the device; requests that arrive while
// others run are admitted as soon as memory and slots free up and form the
// next batches.  Each member's arithmetic depends only on its own data, so a
// request's result does not depend on which batch it ran in.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>

#include "handle.hpp"

namespace {

using Clock = std::chrono::steady_clock;

struct Request {
    uint64_t ticket = 0;
    sg_problem prob{};
    sg_options opt{};
    std::vector<double> target, kappa;
    double* x_out = nullptr;
    size_t footprint = 0;
    Clock::time_point t_submit;
    int state = 0;          // 0 queued, 1 running, 2 done, 3 cancelled
    int status = SG_PENDING;
    int joined = 0;         // 1: took a finished member's slot in a running batch
    sg_solve_info info{};
};

size_t footprint_bytes(const sg_problem& p, const sg_options& o) {
    const double nxi = sg::binom(p.M + p.P, p.P);
    const double nodes = (double)(p.n + 1) * (p.n + 1);
    const double blk = nxi * nodes;
    const double N = 3 * blk;
    const int m = o.restart;
    const bool refine = o.precision == SG_PREC_FP32_REFINE;
    const bool v32 = refine && o.basis_fp32 && o.arnoldi == SG_ARNOLDI_DCGS2;
    const double sz = o.precision == SG_PREC_FP64 ? 8.0 : 4.0;       // Z and preconditioner scratch
    double bytes = (v32 ? 4.0 : 8.0) * N * (m + 1) + sz * N * m;      // basis V, preconditioned vectors Z
    bytes += 8.0 * N * (v32 ? 5 : 6);                                 // FP64 b, x, r (+ w), refinement r, d
    // preconditioner scratch: Schur 2 blocks, hGS 1; multigrid for the widest degree level (~0.6 n_xi
    // columns): restricted right-hand sides, post-smoothed and stored pre-smoothed iterates, about 2 node
    // passes per column over the levels, counted as 4 x 1.4
    bytes += sz * blk * 3 + sz * 4 * nodes * 1.4 * nxi * 0.6;
    if (refine) bytes += 4.0 * N * (v32 ? 2 : 3);                      // FP32 operator output and staging
    if (o.precision == SG_PREC_FP32_PRECOND) bytes += 4.0 * N + 8.0 * N;   // FP32 staging, FP64 copy of Z_j
    // scratch of the preconditioner options: hGSoc level right-hand sides and
    // adjoint intermediates, Richardson iterates, sine-transform solves (FP64)
    if (o.precond == SG_PRECOND_HGSOC) bytes += sz * blk * 4;
    if (o.richardson_steps > 1) bytes += sz * blk * 4;
    if (o.cheb_steps == 0 || o.mean_solver == SG_MEAN_EXACT) bytes += 8.0 * 2 * 2 * blk;
    if (p.field == SG_FIELD_LOGNORMAL) {
        // element coupling tables (all terms, and the truncated ones) and the KKT stiffness scratch
        bytes += 8.0 * (double)p.n * p.n * nxi * nxi * (o.truncation_r > 0 ? 2 : 1) + 8.0 * 2 * blk;
    }
    return (size_t)bytes;
}

bool same_shape(const Request& a, const Request& b) {
    return a.prob.n == b.prob.n && a.prob.M == b.prob.M && a.prob.P == b.prob.P && a.prob.field == b.prob.field &&
           a.opt.precision == b.opt.precision &&
           a.opt.restart == b.opt.restart && a.opt.max_iter == b.opt.max_iter && a.opt.rtol == b.opt.rtol &&
           a.opt.cheb_steps == b.opt.cheb_steps && a.opt.truncation_r == b.opt.truncation_r &&
           a.opt.gmg_pre == b.opt.gmg_pre && a.opt.gmg_post == b.opt.gmg_post && a.opt.inner_rtol == b.opt.inner_rtol &&
           a.opt.arnoldi == b.opt.arnoldi && a.opt.basis_fp32 == b.opt.basis_fp32 &&
           a.opt.mean_solver == b.opt.mean_solver && a.opt.richardson_steps == b.opt.richardson_steps &&
           a.opt.precond == b.opt.precond;
}

}  // namespace

struct sg_server {
    int device = 0;
    size_t budget = 0, in_use = 0;
    int max_slots = 0, running_slots = 0;
    int max_batch = 16;
    int nworkers = 4;
    std::mutex mu;
    std::condition_variable cv_sched, cv_work, cv_done;
    std::deque<uint64_t> queue;
    std::map<uint64_t, std::unique_ptr<Request>> reqs;
    std::deque<std::vector<uint64_t>> batches;       // formed, waiting for a worker
    uint64_t next_ticket = 1;
    bool stopping = false;
    int idle_workers = 0;
    std::thread scheduler;
    std::vector<std::thread> workers;
    std::vector<double> latencies;
    Clock::time_point t_first{}, t_last{};
    bool have_first = false;
    std::string worker_error;
    sg::DevicePool pool;    // device memory of every batch handle (freed when the server is deleted, after the workers joined)

    void schedule_loop();
    void worker_loop(int id);
    void run_batch(const std::vector<uint64_t>& ids, hipStream_t st);
    // completion of request r (lock held)
    void finish(Request& r, const sg_solve_info& info, int status, Clock::time_point now);
};

namespace {

// The member slots of one running batch.  At each restart boundary a slot
// whose request has ended is reported (done) and handed to the oldest queued
// request of the batch's shape (next), which starts from x = 0 in that slot;
// same shape means the same footprint, so the memory budget is unchanged.
struct BatchFeed : sg::SlotFeed {
    sg_server* srv;
    Request shape;                  // n, M, P and options of the batch
    std::vector<uint64_t> slot;     // request in each slot (0: free)

    BatchFeed(sg_server* s, const std::vector<uint64_t>& ids) : srv(s), slot(ids) {
        const Request& r0 = *s->reqs[ids[0]];
        shape.prob = r0.prob;
        shape.opt = r0.opt;
    }
    void done(int q, const double* x_member, const sg_solve_info& info, hipStream_t st) override {
        double* dst;
        size_t n;
        {
            std::lock_guard<std::mutex> lk(srv->mu);
            Request& r = *srv->reqs[slot[q]];
            dst = r.x_out;
            n = (size_t)3 * sg::binom(r.prob.M + r.prob.P, r.prob.P) * (r.prob.n + 1) * (r.prob.n + 1);
        }
        SG_HIP(hipMemcpyAsync(dst, x_member, sizeof(double) * n, hipMemcpyDeviceToHost, st));
        SG_HIP(hipStreamSynchronize(st));
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->finish(*srv->reqs[slot[q]], info, info.status, Clock::now());
    }
    bool next(int q, sg_problem& p) override {
        std::lock_guard<std::mutex> lk(srv->mu);
        if (slot[q]) {      // release the reported request's slot and memory
            srv->in_use -= srv->reqs[slot[q]]->footprint;
            srv->running_slots -= 1;
            slot[q] = 0;
        }
        for (auto it = srv->queue.begin(); it != srv->queue.end(); ++it) {
            Request& r = *srv->reqs[*it];
            if (r.state != 0 || !same_shape(r, shape)) continue;
            if (srv->running_slots >= srv->max_slots || srv->in_use + r.footprint > srv->budget) break;
            r.state = 1;
            r.joined = 1;
            srv->in_use += r.footprint;
            srv->running_slots += 1;
            slot[q] = r.ticket;
            srv->queue.erase(it);
            p = r.prob;
            return true;
        }
        srv->cv_sched.notify_all();
        return false;
    }
};

}  // namespace

void sg_server::finish(Request& r, const sg_solve_info& info, int status, Clock::time_point now) {
    r.info = info;
    r.info.status = status;
    r.info.latency_ms = std::chrono::duration<double, std::milli>(now - r.t_submit).count();
    r.info.joined_batch = r.joined;
    r.status = status;
    r.state = 2;
    latencies.push_back(r.info.latency_ms);
    t_last = now;
    // release the host copies of the inputs
    r.target.clear();
    r.target.shrink_to_fit();
    r.kappa.clear();
    r.kappa.shrink_to_fit();
    cv_done.notify_all();
}

void sg_server::schedule_loop() {
    std::unique_lock<std::mutex> lk(mu);
    while (true) {
        cv_sched.wait(lk, [&] { return stopping || (!queue.empty() && idle_workers > (int)batches.size()); });
        if (stopping && queue.empty()) break;
        // admit in arrival order while memory and slots allow
        std::vector<uint64_t> admitted;
        while (!queue.empty()) {
            Request& r = *reqs[queue.front()];
            if (r.state == 3) {
                queue.pop_front();
                continue;
            }
            if (running_slots + (int)admitted.size() >= max_slots) break;
            if (in_use + r.footprint > budget) break;
            in_use += r.footprint;
            admitted.push_back(queue.front());
            queue.pop_front();
        }
        if (admitted.empty()) {
            if (stopping) break;
            cv_sched.wait(lk);   // wait for memory or slots to free up
            continue;
        }
        // group by shape (stable, arrival order inside a group), cap batch size
        std::vector<bool> used(admitted.size(), false);
        for (size_t i = 0; i < admitted.size(); ++i) {
            if (used[i]) continue;
            std::vector<uint64_t> group{admitted[i]};
            used[i] = true;
            for (size_t k = i + 1; k < admitted.size() && (int)group.size() < max_batch; ++k)
                if (!used[k] && same_shape(*reqs[admitted[i]], *reqs[admitted[k]])) {
                    group.push_back(admitted[k]);
                    used[k] = true;
                }
            for (uint64_t id : group) reqs[id]->state = 1;
            running_slots += (int)group.size();
            batches.push_back(std::move(group));
        }
        cv_work.notify_all();
    }
}

void sg_server::run_batch(const std::vector<uint64_t>& ids, hipStream_t st) {
    std::vector<sg_problem> probs;
    sg_options opt;
    std::unique_ptr<BatchFeed> feed;
    {
        std::lock_guard<std::mutex> lk(mu);
        for (uint64_t id : ids) probs.push_back(reqs[id]->prob);
        opt = reqs[ids[0]]->opt;
        feed = std::make_unique<BatchFeed>(this, ids);
    }
    // Batches run without per-iteration graphs: workers allocate while other
    // workers would be capturing.
    opt.use_graphs = 0;
    const int B = (int)ids.size();
    int code = SG_OK;
    std::string msg;
    try {
        auto h = sg::build_handle(probs.data(), B, &opt, st, &pool);
        const int64_t N = 3 * h->s.blk;
        double* x = h->ws.get_t<double>("serve_x", (size_t)B * N);
        sg::solve(*h, nullptr, x, nullptr, feed.get());
        SG_HIP(hipStreamSynchronize(st));
    } catch (const sg::Error& e) {
        code = e.code;
        msg = e.what();
    } catch (const std::exception& e) {
        code = SG_ERR_INVALID;
        msg = e.what();
    }
    std::lock_guard<std::mutex> lk(mu);
    if (code != SG_OK) {
        // the requests still in the batch's slots fail with the error
        worker_error = msg;
        const auto now = Clock::now();
        for (uint64_t& id : feed->slot) {
            if (!id) continue;
            Request& r = *reqs[id];
            if (r.state != 2) {
                sg_solve_info info{};
                info.status = code;
                finish(r, info, code, now);
            }
            in_use -= r.footprint;
            running_slots -= 1;
            id = 0;
        }
    }
    cv_sched.notify_all();
    cv_done.notify_all();
}

void sg_server::worker_loop(int) {
    hipStream_t st = nullptr;
    if (hipSetDevice(device) != hipSuccess || hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
        std::lock_guard<std::mutex> lk(mu);
        worker_error = "worker could not create a HIP stream";
        return;
    }
    std::unique_lock<std::mutex> lk(mu);
    while (true) {
        ++idle_workers;
        cv_sched.notify_all();
        cv_work.wait(lk, [&] { return !batches.empty() || (stopping && queue.empty() && running_slots == 0); });
        --idle_workers;
        if (batches.empty()) break;
        std::vector<uint64_t> ids = std::move(batches.front());
        batches.pop_front();
        lk.unlock();
        run_batch(ids, st);
        lk.lock();
    }
    lk.unlock();
    (void)hipStreamDestroy(st);
}

extern "C" {

int sg_server_create(size_t hbm_budget_bytes, int32_t max_slots, sg_server** out) {
    try {
        sg::set_last_error("");
        if (!out) throw sg::Error(SG_ERR_INVALID, "out is NULL");
        *out = nullptr;
        if (max_slots < 1 || max_slots > 4096) throw sg::Error(SG_ERR_INVALID, "max_slots must be in [1, 4096]");
        auto s = std::make_unique<sg_server>();
        SG_HIP(hipGetDevice(&s->device));
        if (hbm_budget_bytes == 0) {
            size_t free_b = 0, total_b = 0;
            SG_HIP(hipMemGetInfo(&free_b, &total_b));
            hbm_budget_bytes = (size_t)(0.8 * (double)free_b);
        }
        s->budget = hbm_budget_bytes;
        s->max_slots = max_slots;
        s->max_batch = std::max(1, std::min(16, (int)max_slots));
        sg_server* raw = s.get();
        for (int i = 0; i < s->nworkers; ++i) s->workers.emplace_back([raw, i] { raw->worker_loop(i); });
        s->scheduler = std::thread([raw] { raw->schedule_loop(); });
        *out = s.release();
        return SG_OK;
    } catch (const sg::Error& e) {
        sg::set_last_error(e.what());
        return e.code;
    } catch (...) {
        sg::set_last_error("unknown failure in sg_server_create");
        return SG_ERR_INVALID;
    }
}

int sg_submit(sg_server* s, const sg_problem* prob, const sg_options* opt, double* x_out, uint64_t* ticket) {
    try {
        sg::set_last_error("");
        if (!s || !prob || !x_out || !ticket) throw sg::Error(SG_ERR_INVALID, "null argument");
        sg_options o;
        if (opt)
            o = *opt;
        else
            sg::default_options(&o);
        sg::validate(prob, 1, &o);
        if (prob->n_t >= 2) throw sg::Error(SG_ERR_INVALID, "the server takes steady problems only");
        auto r = std::make_unique<Request>();
        r->prob = *prob;
        r->opt = o;
        const size_t nodes = (size_t)(prob->n + 1) * (prob->n + 1);
        r->target.assign(prob->y_target, prob->y_target + nodes);
        r->prob.y_target = r->target.data();
        if (prob->kappa) {
            r->kappa.assign(prob->kappa, prob->kappa + (size_t)(prob->M + 1) * prob->n * prob->n);
            r->prob.kappa = r->kappa.data();
        }
        r->prob.y0 = nullptr;
        r->x_out = x_out;
        r->footprint = footprint_bytes(*prob, o);
        r->t_submit = Clock::now();
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stopping) throw sg::Error(SG_ERR_INVALID, "server is shutting down");
        if (r->footprint > s->budget)
            throw sg::Error(SG_ERR_NOMEM, "request footprint " + std::to_string(r->footprint) +
                                              " bytes exceeds the server budget");
        r->ticket = s->next_ticket++;
        *ticket = r->ticket;
        if (!s->have_first) {
            s->t_first = r->t_submit;
            s->have_first = true;
        }
        s->queue.push_back(r->ticket);
        s->reqs[r->ticket] = std::move(r);
        s->cv_sched.notify_all();
        return SG_OK;
    } catch (const sg::Error& e) {
        sg::set_last_error(e.what());
        return e.code;
    } catch (...) {
        sg::set_last_error("unknown failure in sg_submit");
        return SG_ERR_INVALID;
    }
}

int sg_poll(sg_server* s, uint64_t ticket, sg_solve_info* info) {
    if (!s) return SG_ERR_INVALID;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return SG_ERR_UNKNOWN;
    Request& r = *it->second;
    if (r.state == 3) return SG_ERR_CANCELLED;
    if (r.state != 2) return SG_PENDING;
    if (info) *info = r.info;
    return r.status;
}

int sg_cancel(sg_server* s, uint64_t ticket) {
    if (!s) return SG_ERR_INVALID;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return SG_ERR_UNKNOWN;
    Request& r = *it->second;
    if (r.state != 0) return SG_ERR_INVALID;
    r.state = 3;
    r.status = SG_ERR_CANCELLED;
    return SG_OK;
}

int sg_server_stats(sg_server* s, int64_t* completed, double* p50_ms, double* p99_ms, double* solves_per_s) {
    if (!s) return SG_ERR_INVALID;
    std::lock_guard<std::mutex> lk(s->mu);
    std::vector<double> l = s->latencies;
    std::sort(l.begin(), l.end());
    auto pct = [&](double q) {
        if (l.empty()) return 0.0;
        const double pos = q * (l.size() - 1);
        const size_t i = (size_t)pos;
        const double f = pos - i;
        return i + 1 < l.size() ? l[i] * (1 - f) + l[i + 1] * f : l[i];
    };
    if (completed) *completed = (int64_t)l.size();
    if (p50_ms) *p50_ms = pct(0.50);
    if (p99_ms) *p99_ms = pct(0.99);
    if (solves_per_s) {
        const double sec = s->have_first ? std::chrono::duration<double>(s->t_last - s->t_first).count() : 0.0;
        *solves_per_s = sec > 0 ? l.size() / sec : 0.0;
    }
    return SG_OK;
}

void sg_server_destroy(sg_server* s) {
    if (!s) return;
    {
        std::unique_lock<std::mutex> lk(s->mu);
        s->cv_done.wait(lk, [&] {
            bool busy = s->running_slots > 0 || !s->batches.empty();
            for (uint64_t id : s->queue)
                if (s->reqs[id]->state == 0) busy = true;
            return !busy;
        });
        s->stopping = true;
        s->cv_sched.notify_all();
        s->cv_work.notify_all();
    }
    if (s->scheduler.joinable()) s->scheduler.join();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->cv_work.notify_all();
    }
    for (auto& w : s->workers)
        if (w.joinable()) w.join();
    delete s;
}

}  // extern "C"
