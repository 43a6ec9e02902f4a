// serve.cpp -- request server with continuous batching (the qp_server_* calls).
//
// One scheduler thread owns the batch lanes.  Each lane is a non-blocking
// stream on which at most one batched launch (one workgroup per instance)
// runs; when a lane's launch completes, the scheduler copies its results out
// and gives the lane the requests that arrived meanwhile, so new work starts
// while the other lanes' launches are still running.  A launch ends with its
// slowest instance, so lanes come in two classes: instances with the
// closed-form primal step (diagonal or zero Q, a few microseconds per
// iteration) and instances with an inner solve (non-diagonal Q), each with
// its own queue, so fast requests never wait behind slow ones.  Requests too
// large for one workgroup go to worker threads that solve them one at a time
// on the single-problem path (each handle has its own stream); these workers
// come in the same two classes, and the diagonal-Q workers never take an
// inner-solve request, so a fast single-path request (a large portfolio)
// does not queue behind slow ones either.  Admission is by
// device bytes: a request starts only when the bytes of everything in flight
// plus its own stay within the budget; the waiting queue is first come,
// first served within each route.
#include <hip/hip_runtime.h>

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

#include "host_internal.h"

using namespace pdhcg;

namespace {

struct Request {
    int64_t id = 0, n = 0, m = 0;
    bool has_q = false;
    std::vector<int64_t> qp, ap;
    std::vector<int32_t> qj, aj;
    std::vector<double> qv, av, c, b, lb, ub;
    std::vector<char> sense;
    size_t bytes = 0;
    int route = 0;   // 0 batched, 1 single path
    int klass = 0;   // batched class: 0 closed form, 1 inner solve
    double t_submit = 0.0;
    // outcome
    int state = 0;   // 0 waiting, 1 running, 2 finished
    int rc = 0;      // status (> 0) or error code (< 0)
    std::vector<double> x, y;
    qp_info info{};
    qp_request_times times{};
};

// Device bytes a request holds while it runs (an upper estimate of what the
// batched or single-problem path allocates for it).
size_t footprint(const Request& r, int route)
{
    const size_t a = (size_t)r.ap[r.m];
    const size_t q = r.has_q ? (size_t)r.qp[r.n] : 0;
    const size_t n = (size_t)r.n, m = (size_t)r.m;
    if (route == 0) {
        // A and A' (values, FP32 copies, columns), Q likewise, row pointers,
        // 18 vectors of n and 10 of m doubles (state, data, power iteration)
        return 16 * (2 * a + q) + 4 * (2 * n + m + 3) + 8 * (18 * n + 10 * m) + 512;
    }
    // single path: CSR of A, A', Q with FP32 copies, schedule descriptors,
    // column-part partial sums, state vectors, control block
    return 16 * (2 * a + q) + 4 * (2 * n + m + 3) + 64 * (2 * n + m) / 8 + 8 * 4 * (2 * n + m) +
           8 * 24 * (n + m) + (1 << 20);
}

struct Lane {
    int klass = 0;
    hipStream_t stream = nullptr;
    qp_batch* bt = nullptr;
    std::vector<Request*> reqs;
    size_t bytes = 0;
    double started = 0.0;
};

}  // namespace

struct qp_server {
    qp_server_config cfg{};
    qp_params params{};
    int device = 0;
    double t0 = 0.0;
    std::mutex mu;
    std::condition_variable cv_sched, cv_work, cv_done;
    std::deque<Request*> bq[2], sq[2];   // waiting: per class, batched and single path
    int workers_of[2] = {0, 0};          // single-path workers per class
    std::map<int64_t, std::unique_ptr<Request>> reqs;
    int64_t next_id = 0;
    size_t in_flight = 0;
    bool stop = false;
    std::vector<Lane> lanes;
    std::thread sched;
    std::vector<std::thread> workers;
};

namespace {

double rel(const qp_server* s) { return now_s() - s->t0; }

void finish_request(qp_server* s, Request* r, int rc)
{
    r->rc = rc;
    r->state = 2;
    r->times.finished = rel(s);
}

// pack the lane's requests block-diagonally and start their launch
int launch_lane(qp_server* s, Lane& L)
{
    const size_t cnt = L.reqs.size();
    std::vector<int64_t> voff(cnt + 1, 0), roff(cnt + 1, 0);
    int64_t qnnz = 0, annz = 0;
    for (size_t i = 0; i < cnt; ++i) {
        const Request* r = L.reqs[i];
        voff[i + 1] = voff[i] + r->n;
        roff[i + 1] = roff[i] + r->m;
        qnnz += r->has_q ? r->qp[r->n] : 0;
        annz += r->ap[r->m];
    }
    const int64_t n = voff[cnt], m = roff[cnt];
    std::vector<int64_t> Qp(n + 1, 0), Ap(m + 1, 0);
    std::vector<int32_t> Qj((size_t)qnnz), Aj((size_t)annz);
    std::vector<double> Qv((size_t)qnnz), Av((size_t)annz), c(n), b(m), lb(n), ub(n);
    std::vector<char> sense(m);
    int64_t qk = 0, ak = 0;
    for (size_t i = 0; i < cnt; ++i) {
        const Request* r = L.reqs[i];
        const int64_t v0 = voff[i], r0 = roff[i];
        for (int64_t j = 0; j < r->n; ++j) {
            if (r->has_q)
                for (int64_t k = r->qp[j]; k < r->qp[j + 1]; ++k) {
                    Qj[qk] = (int32_t)(r->qj[k] + v0);
                    Qv[qk] = r->qv[k];
                    ++qk;
                }
            Qp[v0 + j + 1] = qk;
        }
        for (int64_t j = 0; j < r->m; ++j) {
            for (int64_t k = r->ap[j]; k < r->ap[j + 1]; ++k) {
                Aj[ak] = (int32_t)(r->aj[k] + v0);
                Av[ak] = r->av[k];
                ++ak;
            }
            Ap[r0 + j + 1] = ak;
        }
        std::copy(r->c.begin(), r->c.end(), c.begin() + v0);
        std::copy(r->lb.begin(), r->lb.end(), lb.begin() + v0);
        std::copy(r->ub.begin(), r->ub.end(), ub.begin() + v0);
        std::copy(r->b.begin(), r->b.end(), b.begin() + r0);
        std::copy(r->sense.begin(), r->sense.end(), sense.begin() + r0);
    }
    qp_batch* bt = nullptr;
    int rc = batch_create(L.stream, (int64_t)cnt, voff.data(), roff.data(), Qp.data(), Qj.data(), Qv.data(),
                          Ap.data(), Aj.data(), Av.data(), c.data(), b.data(), sense.data(), lb.data(),
                          ub.data(), &bt);
    if (rc) return rc;
    // each lane class has its own launch shape (a request's result depends
    // only on its class, never on the requests it shares a launch with)
    const int shape = L.klass == 0 ? s->cfg.batch_shape
                                   : (s->cfg.general_shape >= 0 ? s->cfg.general_shape : qp_batch_default_shape(1));
    rc = qp_batch_set_schedule(bt, shape, s->cfg.batch_order);
    if (rc == 0) rc = batch_launch(bt, &s->params);
    if (rc) {
        qp_batch_destroy(bt);
        return rc;
    }
    L.bt = bt;
    return 0;
}

// a lane's launch has ended (pr = 1) or failed (pr < 0): results out, lane free
void complete_lane(qp_server* s, Lane& L, int pr, std::unique_lock<std::mutex>& lk)
{
    std::vector<double> x, y;
    int rc = pr < 0 ? pr : batch_finish(L.bt);
    if (rc >= 0) rc = batch_results_all(L.bt, x, y);
    std::vector<qp_info> infos(L.reqs.size());
    if (rc >= 0)
        for (size_t i = 0; i < L.reqs.size(); ++i) batch_info(L.bt, (int64_t)i, &infos[i]);
    qp_batch_destroy(L.bt);
    L.bt = nullptr;
    lk.lock();
    int64_t v0 = 0, r0 = 0;
    for (size_t i = 0; i < L.reqs.size(); ++i) {
        Request* r = L.reqs[i];
        if (rc >= 0) {
            r->x.assign(x.begin() + v0, x.begin() + v0 + r->n);
            r->y.assign(y.begin() + r0, y.begin() + r0 + r->m);
            r->info = infos[i];
            finish_request(s, r, infos[i].status);
        } else {
            finish_request(s, r, rc);
        }
        v0 += r->n;
        r0 += r->m;
    }
    s->in_flight -= L.bytes;
    L.reqs.clear();
    L.bytes = 0;
    s->cv_done.notify_all();
    s->cv_work.notify_all();
}

void scheduler(qp_server* s)
{
    (void)hipSetDevice(s->device);
    const double linger = s->cfg.batch_linger_us * 1e-6;
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        // completions (device calls without the lock)
        bool running = false;
        for (Lane& L : s->lanes) {
            if (!L.bt) continue;
            lk.unlock();
            const int pr = batch_poll(L.bt);
            if (pr != 0) {
                complete_lane(s, L, pr, lk);   // returns with the lock held
            } else {
                lk.lock();
            }
            running |= L.bt != nullptr;
        }
        if (s->stop && !running) break;
        // admissions
        double wake = -1.0;   // > 0: seconds until the oldest request's linger ends
        if (!s->stop) {
            for (Lane& L : s->lanes) {
                std::deque<Request*>& q = s->bq[L.klass];
                if (L.bt || q.empty()) continue;
                const double age = now_s() - q.front()->t_submit;
                if ((int64_t)q.size() < s->cfg.max_batch && age < linger) {
                    const double wl = linger - age;
                    wake = wake > 0.0 ? std::min(wake, wl) : wl;
                    continue;
                }
                size_t bytes = 0;
                while (!q.empty() && (int64_t)L.reqs.size() < s->cfg.max_batch) {
                    Request* r = q.front();
                    if (s->in_flight + bytes + r->bytes > (size_t)s->cfg.device_budget) break;
                    q.pop_front();
                    L.reqs.push_back(r);
                    bytes += r->bytes;
                }
                if (L.reqs.empty()) continue;   // budget full: wait for completions
                s->in_flight += bytes;
                L.bytes = bytes;
                const double t = rel(s);
                for (Request* r : L.reqs) {
                    r->state = 1;
                    r->times.started = t;
                    r->times.batch_size = (int32_t)L.reqs.size();
                }
                lk.unlock();
                const int rc = launch_lane(s, L);
                lk.lock();
                if (rc) {
                    for (Request* r : L.reqs) finish_request(s, r, rc);
                    s->in_flight -= L.bytes;
                    L.reqs.clear();
                    L.bytes = 0;
                    s->cv_done.notify_all();
                } else {
                    running = true;
                }
            }
        }
        if (running) {
            s->cv_sched.wait_for(lk, std::chrono::microseconds(20));
        } else if (wake > 0.0) {
            s->cv_sched.wait_for(lk, std::chrono::duration<double>(wake));
        } else if (!s->stop) {
            s->cv_sched.wait(lk);
        }
    }
}

// the single-path queue a worker of class k takes its next request from
// (own class first; a general worker helps with diagonal-Q requests, and a
// diagonal-Q worker takes general ones only when there is no general
// worker), or -1 when nothing it may take fits the budget
int pick_queue(const qp_server* s, int k)
{
    auto fits = [&](int q) {
        return !s->sq[q].empty() && s->in_flight + s->sq[q].front()->bytes <= (size_t)s->cfg.device_budget;
    };
    if (fits(k)) return k;
    if ((k == 1 || s->workers_of[1] == 0) && fits(1 - k)) return 1 - k;
    return -1;
}

void worker(qp_server* s, int k)
{
    (void)hipSetDevice(s->device);
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        int q = -1;
        s->cv_work.wait(lk, [&] { return s->stop || (q = pick_queue(s, k)) >= 0; });
        if (s->stop) break;
        Request* r = s->sq[q].front();
        s->sq[q].pop_front();
        s->in_flight += r->bytes;
        r->state = 1;
        r->times.started = rel(s);
        r->times.batch_size = 1;
        lk.unlock();
        qp_handle* h = nullptr;
        int rc = qp_create(r->n, r->m, r->has_q ? r->qp.data() : nullptr, r->qj.data(), r->qv.data(),
                           r->ap.data(), r->aj.data(), r->av.data(), r->c.data(), r->b.data(),
                           r->sense.data(), r->lb.data(), r->ub.data(), &h);
        if (rc == 0) rc = qp_solve_ex(h, &s->params);
        std::vector<double> x(r->n), y(r->m);
        qp_info info{};
        if (rc > 0) {
            const int rr = qp_result(h, x.data(), y.data(), &info);
            if (rr < 0) rc = rr;
        }
        if (h) qp_destroy(h);
        lk.lock();
        r->x.swap(x);
        r->y.swap(y);
        r->info = info;
        finish_request(s, r, rc);
        s->in_flight -= r->bytes;
        s->cv_done.notify_all();
        s->cv_work.notify_all();
        s->cv_sched.notify_all();
    }
}

}  // namespace

extern "C" {

qp_server_config qp_server_config_default(void)
{
    qp_server_config c{};
    c.device_budget = (int64_t)8 << 30;
    c.batch_max_dim = 20000;
    c.general_max_dim = 3000;
    c.batch_lanes = 2;
    c.general_lanes = 2;
    c.single_workers = 5;
    c.max_batch = 1024;
    c.batch_shape = -1;
    c.batch_order = -1;
    c.general_shape = -1;
    c.diag_workers = -1;
    c.batch_linger_us = 200.0;
    return c;
}

int qp_server_create(const qp_server_config* cfg, const qp_params* params, qp_server** out)
{
    if (!out) return fail(QP_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    const qp_server_config c = cfg ? *cfg : qp_server_config_default();
    const qp_params p = params ? *params : qp_params_default();
    if (c.device_budget <= 0 || c.batch_max_dim < 0 || c.general_max_dim < 0 || c.batch_lanes < 0 ||
        c.general_lanes < 0 || c.single_workers < 0 || c.batch_lanes + c.general_lanes + c.single_workers < 1 ||
        c.max_batch < 1 || !(c.batch_linger_us >= 0.0) || c.batch_shape < -1 ||
        c.batch_shape >= qp_batch_num_shapes() || c.batch_order < -1 || c.batch_order > 1 ||
        c.general_shape < -1 || c.general_shape >= qp_batch_num_shapes() || c.diag_workers < -1 ||
        c.diag_workers > c.single_workers)
        return fail(QP_ERR_INVALID_ARG, "invalid server configuration");
    if (!(p.tol > 0.0) || p.max_iter < 0 || p.check_every < 1 ||
        (p.precision != QP_PRECISION_FP64 && p.precision != QP_PRECISION_MIXED))
        return fail(QP_ERR_INVALID_ARG, "invalid parameters");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return fail(QP_ERR_DEVICE, "no HIP device available");
    qp_server* s = new qp_server();
    s->cfg = c;
    s->params = p;
    s->params.timing = 0;
    s->t0 = now_s();
    if (hipGetDevice(&s->device) != hipSuccess) {
        delete s;
        return fail(QP_ERR_DEVICE, "hipGetDevice failed");
    }
    s->lanes.resize((size_t)(c.batch_lanes + c.general_lanes));
    for (int i = 0; i < c.batch_lanes + c.general_lanes; ++i) s->lanes[i].klass = i < c.batch_lanes ? 0 : 1;
    for (Lane& L : s->lanes) {
        if (hipStreamCreateWithFlags(&L.stream, hipStreamNonBlocking) != hipSuccess) {
            for (Lane& K : s->lanes)
                if (K.stream) (void)hipStreamDestroy(K.stream);
            delete s;
            return fail(QP_ERR_DEVICE, "hipStreamCreate failed");
        }
    }
    if (c.batch_lanes + c.general_lanes > 0) s->sched = std::thread(scheduler, s);
    s->workers_of[0] = c.diag_workers >= 0 ? c.diag_workers : (c.single_workers >= 2 ? 1 : 0);
    s->workers_of[1] = c.single_workers - s->workers_of[0];
    for (int i = 0; i < c.single_workers; ++i) s->workers.emplace_back(worker, s, i < s->workers_of[0] ? 0 : 1);
    *out = s;
    return 0;
}

int64_t qp_server_submit(qp_server* s, int64_t n, int64_t m,
                         const int64_t* Qp, const int32_t* Qj, const double* Qv,
                         const int64_t* Ap, const int32_t* Aj, const double* Av,
                         const double* c, const double* b, const char* sense,
                         const double* lb, const double* ub)
{
    if (!s) return fail(QP_ERR_INVALID_ARG, "server is NULL");
    const double t_submit = now_s();
    if (n < 1 || m < 0 || n >= INT32_MAX || m >= INT32_MAX) return fail(QP_ERR_INVALID_ARG, "need n >= 1, m >= 0");
    int rc;
    std::vector<int64_t> a_empty(1, 0);
    if (!Ap) {
        if (m != 0) return fail(QP_ERR_INVALID_ARG, "A: row pointer is NULL");
        Ap = a_empty.data();
    }
    if ((rc = check_csr("A", m, n, Ap, Aj, Av))) return rc;
    if (Qp) {
        if ((rc = check_csr("Q", n, n, Qp, Qj, Qv))) return rc;
        if ((rc = check_symmetric(n, Qp, Qj, Qv))) return rc;
    }
    if ((rc = check_vec("c", n, c, false))) return rc;
    if (m > 0) {
        if (!b || !sense) return fail(QP_ERR_INVALID_ARG, "b or sense is NULL");
        if ((rc = check_vec("b", m, b, false))) return rc;
        for (int64_t i = 0; i < m; ++i)
            if (sense[i] != 'E' && sense[i] != 'G' && sense[i] != 'L')
                return fail(QP_ERR_INVALID_ARG, "sense must be 'E', 'G' or 'L'");
    }
    auto r = std::make_unique<Request>();
    r->n = n;
    r->m = m;
    r->has_q = Qp != nullptr;
    r->lb.resize(n);
    r->ub.resize(n);
    for (int64_t i = 0; i < n; ++i) {
        r->lb[i] = lb ? lb[i] : -INFINITY;
        r->ub[i] = ub ? ub[i] : INFINITY;
    }
    if ((rc = check_bounds("lb/ub", n, r->lb.data(), r->ub.data()))) return rc;
    r->ap.assign(Ap, Ap + m + 1);
    r->aj.assign(Aj, Aj + Ap[m]);
    r->av.assign(Av, Av + Ap[m]);
    if (Qp) {
        r->qp.assign(Qp, Qp + n + 1);
        r->qj.assign(Qj, Qj + Qp[n]);
        r->qv.assign(Qv, Qv + Qp[n]);
    } else {
        r->qp.assign(n + 1, 0);
    }
    r->c.assign(c, c + n);
    if (m > 0) {
        r->b.assign(b, b + m);
        r->sense.assign(sense, sense + m);
    }
    // the batched kernel sums each row with one thread: a long row (a budget
    // row over every asset, a dense column of A) would serialise its instance
    int64_t longest = 0;
    for (int64_t i = 0; i < m; ++i) longest = std::max(longest, Ap[i + 1] - Ap[i]);
    if (Qp)
        for (int64_t i = 0; i < n; ++i) longest = std::max(longest, Qp[i + 1] - Qp[i]);
    {
        std::vector<int64_t> colcnt(n, 0);
        for (int64_t e = 0; e < Ap[m]; ++e) ++colcnt[Aj[e]];
        for (int64_t i = 0; i < n; ++i) longest = std::max(longest, colcnt[i]);
    }
    bool diagonal = true;
    if (Qp)
        for (int64_t i = 0; i < n && diagonal; ++i)
            for (int64_t e = Qp[i]; e < Qp[i + 1]; ++e)
                if (Qj[e] != i) { diagonal = false; break; }
    r->klass = diagonal ? 0 : 1;
    const int64_t lanes = diagonal ? s->cfg.batch_lanes : s->cfg.general_lanes;
    const int64_t limit = diagonal ? s->cfg.batch_max_dim : s->cfg.general_max_dim;
    const bool small = n + m <= limit && longest <= QP_BATCH_MAX_ROW;
    if (lanes > 0 && (small || s->cfg.single_workers == 0)) r->route = 0;
    else if (s->cfg.single_workers > 0) r->route = 1;
    else return fail(QP_ERR_INVALID_ARG, "no lane or worker takes this request");
    r->bytes = footprint(*r, r->route);
    if (r->bytes > (size_t)s->cfg.device_budget) return fail(QP_ERR_INVALID_ARG, "request exceeds the device budget");
    r->t_submit = t_submit;
    r->times.route = r->route;
    Request* raw = r.get();
    std::lock_guard<std::mutex> g(s->mu);
    if (s->stop) return fail(QP_ERR_STATE, "server is stopping");
    raw->id = s->next_id++;
    raw->times.submitted = t_submit - s->t0;
    s->reqs.emplace(raw->id, std::move(r));
    if (raw->route == 0) {
        s->bq[raw->klass].push_back(raw);
        s->cv_sched.notify_one();
    } else {
        s->sq[raw->klass].push_back(raw);
        s->cv_work.notify_all();
    }
    g_err.clear();
    return raw->id;
}

int qp_server_wait(qp_server* s, int64_t id, double timeout_s)
{
    if (!s) return fail(QP_ERR_INVALID_ARG, "server is NULL");
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(id);
    if (it == s->reqs.end()) return fail(QP_ERR_INVALID_ARG, "unknown request id");
    Request* r = it->second.get();
    auto ready = [&] { return r->state == 2; };
    if (timeout_s < 0.0) s->cv_done.wait(lk, ready);
    else if (!s->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), ready)) return QP_NOT_SOLVED;
    if (r->rc < 0) return fail(r->rc, "the request's solve failed");
    return r->rc;
}

int qp_server_result(qp_server* s, int64_t id, double* x, double* y, qp_info* info, qp_request_times* times)
{
    if (!s) return fail(QP_ERR_INVALID_ARG, "server is NULL");
    std::unique_ptr<Request> r;
    {
        std::lock_guard<std::mutex> g(s->mu);
        auto it = s->reqs.find(id);
        if (it == s->reqs.end()) return fail(QP_ERR_INVALID_ARG, "unknown request id");
        if (it->second->state != 2) return fail(QP_ERR_STATE, "request not finished");
        r = std::move(it->second);
        s->reqs.erase(it);
    }
    if (x && !r->x.empty()) std::copy(r->x.begin(), r->x.end(), x);
    if (y && !r->y.empty()) std::copy(r->y.begin(), r->y.end(), y);
    if (info) *info = r->info;
    if (times) *times = r->times;
    return r->rc;
}

void qp_server_destroy(qp_server* s)
{
    if (!s) return;
    {
        std::lock_guard<std::mutex> g(s->mu);
        s->stop = true;
        s->bq[0].clear();
        s->bq[1].clear();
        s->sq[0].clear();
        s->sq[1].clear();
    }
    s->cv_sched.notify_all();
    s->cv_work.notify_all();
    if (s->sched.joinable()) s->sched.join();
    for (std::thread& t : s->workers)
        if (t.joinable()) t.join();
    for (Lane& L : s->lanes)
        if (L.stream) (void)hipStreamDestroy(L.stream);
    delete s;
}

}  // extern "C"
