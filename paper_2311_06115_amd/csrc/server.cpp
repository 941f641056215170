// Serving loop: diffusion-map eigensolves of different sizes arrive while
// others run.  Requests are admitted by free slots and by their estimated
// device-memory footprint (first come, first served); a compressor thread
// builds each admitted request's operator on its own stream while the solver
// thread advances every running eigensolve by one Lanczos step per tick, with
// the products of all running solves that share a tile precision issued as one
// launch per phase.  Each solve's arithmetic is the same as when it runs alone.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "op.hpp"

namespace {

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct ServeReq {
    uint64_t ticket = 0;
    hdm_params prm{};
    std::vector<uint8_t> X;      // host copy taken at submission
    int r = 0;
    double tol = 0.0;
    int max_basis = 0;
    double arrival_s = 0.0, admit_s = 0.0, done_s = 0.0;
    enum State { QUEUED, ADMITTED, SOLVING, DONE } state = QUEUED;
    bool cancel = false;
    size_t est = 0;              // admission footprint
    size_t held = 0;             // bytes accounted while admitted
    std::unique_ptr<hdm_op_s> op;
    hdm::LanczosRun run;
    hdm_result_t res{};
};

using ReqPtr = std::shared_ptr<ServeReq>;

}  // namespace

struct hdm_server_s {
    hdm_ctx ctx = nullptr;
    hdm_server_cfg_t cfg{};
    std::mutex mu;
    std::condition_variable cv;
    std::map<uint64_t, ReqPtr> all;
    std::deque<ReqPtr> queue;          // waiting for admission
    std::deque<ReqPtr> to_compress;    // admitted, waiting for the compressor
    std::vector<ReqPtr> ready;         // compressed, to be picked up by the solver
    int active = 0;                    // admitted and not finished
    size_t resident = 0, peak = 0;
    uint64_t next_ticket = 1;
    bool stop = false;
    // statistics
    int64_t submitted = 0, admitted = 0, completed = 0, rejected = 0, cancelled = 0, shared = 0;
    std::vector<double> latencies;
    double first_arrival = 0.0, last_done = 0.0;
    std::thread solver;
    std::vector<std::thread> compressors;
};

namespace {

// finish a request (lock held): release its memory and record its outcome;
// a request is finished once
void finish_locked(hdm_server_s* S, const ReqPtr& q, int status) {
    if (q->state == ServeReq::DONE) return;
    q->done_s = now_s();
    q->res.status = status;
    q->res.latency_s = q->done_s - q->arrival_s;
    q->res.service_s = q->admit_s > 0.0 ? q->done_s - q->admit_s : 0.0;
    q->X.clear();
    q->X.shrink_to_fit();
    q->res.x_released = 1;
    if (q->state != ServeReq::QUEUED) {
        S->active -= 1;
        S->resident -= std::min(S->resident, q->held);
    }
    q->held = 0;
    q->state = ServeReq::DONE;
    if (status == HDM_OK || status == HDM_ENOCONV) {
        S->completed += 1;
        S->latencies.push_back(q->res.latency_s);
        S->last_done = std::max(S->last_done, q->done_s);
    } else if (status == HDM_ECANCELLED) {
        S->cancelled += 1;
    }
    S->cv.notify_all();
}

// admission in arrival order by free slots and memory (lock held)
void admit_locked(hdm_server_s* S) {
    while (!S->queue.empty() && S->active < S->cfg.max_slots) {
        ReqPtr q = S->queue.front();
        if (S->cfg.mem_budget_bytes && S->resident + q->est > S->cfg.mem_budget_bytes) break;
        S->queue.pop_front();
        q->state = ServeReq::ADMITTED;
        q->admit_s = now_s();
        q->held = q->est;
        S->resident += q->est;
        S->peak = std::max(S->peak, S->resident);
        S->active += 1;
        S->admitted += 1;
        S->to_compress.push_back(q);
    }
    S->cv.notify_all();
}

// frees a request's device state; the release waits for the device at the end
// of the scope (as in hdm_op_destroy) instead of one hipFree per buffer
void release_solve(const ReqPtr& q) {
    hdm::PoolScope pool_scope;
    q->run = hdm::LanczosRun();
    q->op.reset();
}

void compressor_main(hdm_server_s* S) {
    (void)hipSetDevice(S->ctx->device);
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return;
    for (;;) {
        ReqPtr q;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            S->cv.wait(lk, [&] { return S->stop || !S->to_compress.empty(); });
            if (S->stop) break;
            q = S->to_compress.front();
            S->to_compress.pop_front();
            if (q->cancel) {
                finish_locked(S, q, HDM_ECANCELLED);
                admit_locked(S);
                continue;
            }
        }
        int status = HDM_OK;
        try {
            // the same buffer lifetime rules as hdm_compress: releases wait for
            // the device at the end of the scope, uploads go through pinned staging
            hdm::PoolScope pool_scope;
            q->op.reset(hdm::make_operator(S->ctx, q->X.data(), 0, q->prm, s));
            q->run.start(*q->op, q->r, q->tol, q->max_basis, q->prm.seed, s);
            HDM_HIP(hipStreamSynchronize(s));
        } catch (const hdm::Error& e) {
            status = e.code;
        } catch (...) {
            status = HDM_EINTERNAL;
        }
        if (status != HDM_OK) release_solve(q);
        std::lock_guard<std::mutex> lk(S->mu);
        if (status == HDM_OK) {
            // the operator holds its own copy of the points
            q->X.clear();
            q->X.shrink_to_fit();
            q->res.x_released = 1;
        }
        if (status != HDM_OK) {
            finish_locked(S, q, status);
            admit_locked(S);
            continue;
        }
        // replace the estimate by what the request really holds
        const size_t actual = q->op->footprint() + q->run.bytes();
        S->resident = S->resident - std::min(S->resident, q->held) + actual;
        S->peak = std::max(S->peak, S->resident);
        q->held = actual;
        q->state = ServeReq::SOLVING;
        S->ready.push_back(q);
        admit_locked(S);
    }
    (void)hipStreamDestroy(s);
}

void solver_main(hdm_server_s* S) {
    (void)hipSetDevice(S->ctx->device);
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return;
    hdm::Lane lane;
    try {
        lane.init();
    } catch (...) {
        (void)hipStreamDestroy(s);
        return;
    }
    std::vector<ReqPtr> running;
    for (;;) {
        {
            std::unique_lock<std::mutex> lk(S->mu);
            S->cv.wait(lk, [&] { return S->stop || !S->ready.empty() || !running.empty(); });
            if (S->stop) break;
            for (auto& q : S->ready) running.push_back(q);
            S->ready.clear();
            // cancelled solves leave before the tick
            for (auto it = running.begin(); it != running.end();) {
                if ((*it)->cancel) {
                    release_solve(*it);
                    finish_locked(S, *it, HDM_ECANCELLED);
                    it = running.erase(it);
                } else {
                    ++it;
                }
            }
            admit_locked(S);
        }
        if (running.empty()) continue;
        std::vector<ReqPtr> done;
        std::vector<int> done_status;
        try {
            // one product per running solve: groups of equal tile precision, at most kMaxBatch per launch
            std::vector<bool> taken(running.size(), false);
            for (size_t a = 0; a < running.size(); ++a) {
                if (taken[a]) continue;
                std::vector<hdm::ApplyReq> batch;
                for (size_t b = a; b < running.size() && static_cast<int>(batch.size()) < hdm::kMaxBatch; ++b) {
                    if (taken[b]) continue;
                    const hdm_params& pa = running[a]->prm;
                    const hdm_params& pb = running[b]->prm;
                    if (pa.near_prec != pb.near_prec || pa.far_prec != pb.far_prec) continue;
                    taken[b] = true;
                    batch.push_back(hdm::ApplyReq{running[b]->op.get(), running[b]->run.current(),
                                                  running[b]->run.output()});
                }
                hdm::apply_batch(batch.data(), static_cast<int>(batch.size()), 1, 1, s, lane, S->ctx);
                if (batch.size() > 1) {
                    std::lock_guard<std::mutex> lk(S->mu);
                    S->shared += 1;
                }
            }
            for (auto& q : running) {
                if (q->run.after_product(s)) {
                    const hdm_status st = q->run.result(q->res.evals, nullptr, nullptr, s);
                    q->res.r = q->r;
                    q->res.iters = q->run.m;
                    done.push_back(q);
                    done_status.push_back(st);
                }
            }
        } catch (const hdm::Error& e) {
            // a device failure ends every running solve with that status (the
            // ones already finished this tick keep theirs)
            for (auto& q : running) {
                if (std::find(done.begin(), done.end(), q) != done.end()) continue;
                done.push_back(q);
                done_status.push_back(e.code);
            }
        }
        if (!done.empty()) {
            // device state released outside the lock (the release waits for the device)
            {
                hdm::PoolScope one_wait;   // the nested releases wait once, at its end
                for (const ReqPtr& q : done) release_solve(q);
            }
            std::lock_guard<std::mutex> lk(S->mu);
            for (size_t t = 0; t < done.size(); ++t) {
                ReqPtr q = done[t];
                running.erase(std::remove(running.begin(), running.end(), q), running.end());
                finish_locked(S, q, done_status[t]);
            }
            admit_locked(S);
        }
    }
    for (auto& q : running) release_solve(q);
    (void)hipStreamDestroy(s);
}

template <typename F>
hdm_status guarded(F&& f) {
    try {
        hdm::set_last_error("");
        return f();
    } catch (const hdm::Error& e) {
        hdm::set_last_error(e.what());
        return e.code;
    } catch (const std::exception& e) {
        hdm::set_last_error(e.what());
        return HDM_EINTERNAL;
    }
}

}  // namespace

extern "C" {

hdm_status hdm_server_create(hdm_ctx ctx, const hdm_server_cfg_t* cfg, hdm_server* out) {
    return guarded([&] {
        HDM_CHECK(ctx && cfg && out, HDM_EINVAL, "NULL argument");
        HDM_CHECK(cfg->max_slots >= 1 && cfg->max_slots <= 64, HDM_EINVAL, "max_slots must be in [1, 64]");
        HDM_CHECK(cfg->compressors >= 0 && cfg->compressors <= 8, HDM_EINVAL, "compressors must be in [0, 8]");
        auto* S = new hdm_server_s();
        S->ctx = ctx;
        S->cfg = *cfg;
        const int nc = cfg->compressors > 0 ? cfg->compressors : 2;
        for (int t = 0; t < nc; ++t) S->compressors.emplace_back(compressor_main, S);
        S->solver = std::thread(solver_main, S);
        *out = S;
        return HDM_OK;
    });
}

hdm_status hdm_submit(hdm_server S, const hdm_request_t* req, uint64_t* ticket) {
    return guarded([&] {
        HDM_CHECK(S && req && req->X && ticket, HDM_EINVAL, "NULL argument");
        hdm::validate_params(req->params);
        HDM_CHECK(req->r >= 1 && req->r <= 64 && req->r <= req->params.n, HDM_EINVAL, "r must be in [1, min(64, n)]");
        HDM_CHECK(req->rel_resid_tol > 0.0, HDM_EINVAL, "rel_resid_tol must be > 0");
        auto q = std::make_shared<ServeReq>();
        q->prm = req->params;
        const size_t xb = static_cast<size_t>(req->params.n) * req->params.dim * hdm::dtype_size(req->params.x_dtype);
        q->X.assign(static_cast<const uint8_t*>(req->X), static_cast<const uint8_t*>(req->X) + xb);
        if (req->params.x_dtype == HDM_F64) {
            const double* x = reinterpret_cast<const double*>(q->X.data());
            for (size_t i = 0; i < xb / 8; ++i) HDM_CHECK(std::isfinite(x[i]), HDM_EINVAL, "points contain NaN or Inf");
        }
        q->r = req->r;
        q->tol = req->rel_resid_tol;
        q->max_basis = req->max_basis > 0 ? req->max_basis : static_cast<int>(std::min<int64_t>(req->params.n, 300));
        q->arrival_s = req->arrival_s > 0.0 ? req->arrival_s : now_s();
        q->est = hdm::footprint_estimate(req->params, q->max_basis);
        q->res.x_released = 0;   // the host copy is kept until the operator is built
        std::lock_guard<std::mutex> lk(S->mu);
        S->submitted += 1;
        if (S->first_arrival == 0.0 || q->arrival_s < S->first_arrival) S->first_arrival = q->arrival_s;
        if (S->cfg.mem_budget_bytes && q->est > S->cfg.mem_budget_bytes) {
            S->rejected += 1;
            hdm::fail(HDM_ENOMEM, "request footprint exceeds the server's memory budget");
        }
        q->ticket = S->next_ticket++;
        S->all[q->ticket] = q;
        S->queue.push_back(q);
        *ticket = q->ticket;
        admit_locked(S);
        return HDM_OK;
    });
}

hdm_status hdm_poll(hdm_server S, uint64_t ticket, hdm_result_t* out) {
    return guarded([&] {
        HDM_CHECK(S && out, HDM_EINVAL, "NULL argument");
        std::lock_guard<std::mutex> lk(S->mu);
        auto it = S->all.find(ticket);
        HDM_CHECK(it != S->all.end(), HDM_EINVAL, "unknown ticket");
        if (it->second->state != ServeReq::DONE) return HDM_EBUSY;
        *out = it->second->res;
        S->all.erase(it);   // a result is handed out once; the ticket is then unknown
        return HDM_OK;
    });
}

hdm_status hdm_cancel(hdm_server S, uint64_t ticket) {
    return guarded([&] {
        HDM_CHECK(S, HDM_EINVAL, "NULL server");
        std::lock_guard<std::mutex> lk(S->mu);
        auto it = S->all.find(ticket);
        HDM_CHECK(it != S->all.end(), HDM_EINVAL, "unknown ticket");
        ReqPtr q = it->second;
        if (q->state == ServeReq::DONE) return HDM_OK;
        if (q->state == ServeReq::QUEUED) {
            S->queue.erase(std::remove(S->queue.begin(), S->queue.end(), q), S->queue.end());
            finish_locked(S, q, HDM_ECANCELLED);
            return HDM_OK;
        }
        q->cancel = true;   // the worker holding it releases it at its next step
        return HDM_OK;
    });
}

hdm_status hdm_server_stats(hdm_server S, hdm_server_stats_t* out) {
    return guarded([&] {
        HDM_CHECK(S && out, HDM_EINVAL, "NULL argument");
        std::lock_guard<std::mutex> lk(S->mu);
        hdm_server_stats_t st{};
        st.submitted = S->submitted;
        st.admitted = S->admitted;
        st.completed = S->completed;
        st.rejected = S->rejected;
        st.cancelled = S->cancelled;
        st.peak_resident_bytes = static_cast<int64_t>(S->peak);
        st.shared_launches = S->shared;
        if (!S->latencies.empty()) {
            std::vector<double> l = S->latencies;
            std::sort(l.begin(), l.end());
            auto pct = [&](double p) {
                const double pos = p * static_cast<double>(l.size() - 1);
                const size_t lo = static_cast<size_t>(pos);
                const size_t hi = std::min(lo + 1, l.size() - 1);
                return l[lo] + (l[hi] - l[lo]) * (pos - static_cast<double>(lo));
            };
            st.p50_latency_s = pct(0.50);
            st.p99_latency_s = pct(0.99);
            const double span = S->last_done - S->first_arrival;
            st.solves_per_s = span > 0.0 ? static_cast<double>(S->completed) / span : 0.0;
        }
        *out = st;
        return HDM_OK;
    });
}

hdm_status hdm_server_destroy(hdm_server S) {
    return guarded([&] {
        if (!S) return HDM_OK;
        {
            std::lock_guard<std::mutex> lk(S->mu);
            S->stop = true;
            S->cv.notify_all();
        }
        for (auto& t : S->compressors)
            if (t.joinable()) t.join();
        if (S->solver.joinable()) S->solver.join();
        delete S;
        return HDM_OK;
    });
}

}  // extern "C"
