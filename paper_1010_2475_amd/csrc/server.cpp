// Continuous-batching solve server (mmvm_server_* in include/mmvm.h).
//
// A worker thread owns the device side.  Requests wait in a FIFO queue until
// a slot is free and their HBM footprint (state + a private workspace) fits
// the budget; then their state is copied to the device and they join the
// resident set.  Every scheduling round the worker gives each resident request
// a chunk of RK4 steps on one of several HIP streams, so the kernels of
// different requests overlap on the device, and requests that arrive meanwhile
// join at the next round.  A finished request is copied back, its memory and
// slot are released, and its ticket becomes pollable.  Each request has its
// own workspace and state, so its result does not depend on what else is
// resident (bitwise: the kernels are deterministic).
#include <hip/hip_runtime.h>

#include <atomic>
#include <cmath>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "api_internal.hpp"

namespace mmvm {
namespace {

constexpr int kStreams = 4;          // hardware queues per process on the target
constexpr int64_t kChunkSteps = 25;  // RK4 steps per scheduling quantum

enum ReqState { Q_QUEUED, Q_RESIDENT, Q_DONE, Q_FAILED };

struct Request {
    uint64_t ticket = 0;
    int n = 0, order = 0;
    double nu = 0.0, t0 = 0.0, dt = 0.0;
    int64_t nsteps = 0, done_steps = 0, inflight = 0;
    mmvm_precision prec = MMVM_MIXED;
    std::vector<double> lambda0, x, mom;  // host input, then host result
    size_t footprint = 0;
    ReqState state = Q_QUEUED;
    mmvm_status status = MMVM_OK;
    // device side
    int stream = 0;
    double* dx = nullptr;
    double* dmom = nullptr;
    std::unique_ptr<Workspace> ws;
    hipEvent_t ev = nullptr;
    mmvm_stats stats{};
};

size_t state_bytes(int n, int M) { return sizeof(double) * (size_t)n * (2 + (size_t)(M + 1) * (M + 2) / 2); }

}  // namespace
}  // namespace mmvm

using namespace mmvm;

struct mmvm_server {
    size_t budget = 0;
    int max_slots = 0;
    int device = 0;
    std::chrono::steady_clock::time_point t_origin;
    hipStream_t streams[kStreams] = {};

    std::mutex mu;
    std::condition_variable cv_work;  // worker wake-up
    std::condition_variable cv_idle;  // drain
    std::deque<Request*> queue;
    std::vector<Request*> resident;
    std::map<uint64_t, std::unique_ptr<Request>> all;
    size_t used = 0;
    uint64_t next_ticket = 1;
    bool stop = false;
    std::thread worker;

    double now() const
    {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t_origin).count();
    }
    void run();
    bool admit_locked(Request* r);
    void finish(Request* r, mmvm_status st);
};

bool mmvm_server::admit_locked(Request* r)
{
    if ((int)resident.size() >= max_slots || used + r->footprint > budget) return false;
    // allocate and upload (device calls while holding the lock are short and
    // only contend with submit/poll bookkeeping)
    r->stream = (int)(r->ticket % kStreams);
    hipStream_t st = streams[r->stream];
    r->ws.reset(new Workspace());
    mmvm_status s = r->ws->ensure(r->n, r->order, use_dd(r->order, r->prec), r->n == 1, st);
    if (s == MMVM_OK) s = r->ws->set_params(r->lambda0.data(), nullptr, r->nu, r->n, st);
    const size_t sb = state_bytes(r->n, r->order);
    if (s == MMVM_OK && hipMalloc((void**)&r->dx, sb) != hipSuccess) s = MMVM_ENOMEM;
    if (s == MMVM_OK) {
        r->dmom = r->dx + 2 * (size_t)r->n;
        if (hipMemcpyAsync(r->dx, r->x.data(), sizeof(double) * 2 * r->n, hipMemcpyHostToDevice, st) != hipSuccess ||
            hipMemcpyAsync(r->dmom, r->mom.data(), sizeof(double) * r->mom.size(), hipMemcpyHostToDevice, st) !=
                hipSuccess ||
            hipEventCreateWithFlags(&r->ev, hipEventDisableTiming) != hipSuccess)
            s = MMVM_EDEVICE;
    }
    used += r->footprint;
    r->state = Q_RESIDENT;
    r->stats.t_admit = now();
    resident.push_back(r);
    if (s != MMVM_OK) finish(r, s);
    return true;
}

void mmvm_server::finish(Request* r, mmvm_status st)
{
    // caller holds mu
    if (st == MMVM_OK && r->dx) {
        hipStream_t s = streams[r->stream];
        if (hipMemcpyAsync(r->x.data(), r->dx, sizeof(double) * 2 * r->n, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipMemcpyAsync(r->mom.data(), r->dmom, sizeof(double) * r->mom.size(), hipMemcpyDeviceToHost, s) !=
                hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            st = MMVM_EDEVICE;
    }
    if (r->dx) (void)hipFree(r->dx);
    r->dx = r->dmom = nullptr;
    r->ws.reset();
    if (r->ev) (void)hipEventDestroy(r->ev);
    r->ev = nullptr;
    used -= r->footprint;
    r->state = st == MMVM_OK ? Q_DONE : Q_FAILED;
    r->status = st;
    r->stats.t_done = now();
    r->stats.steps = r->done_steps;
    for (size_t i = 0; i < resident.size(); ++i)
        if (resident[i] == r) {
            resident.erase(resident.begin() + (long)i);
            break;
        }
}

void mmvm_server::run()
{
    (void)hipSetDevice(device);
    std::unique_lock<std::mutex> lk(mu);
    while (true) {
        // admit in arrival order while slots and memory allow
        while (!queue.empty() && admit_locked(queue.front())) queue.pop_front();
        if (stop && queue.empty() && resident.empty()) break;
        if (resident.empty()) {
            cv_idle.notify_all();
            if (stop) break;
            cv_work.wait(lk);
            continue;
        }
        // give every idle resident request its next chunk
        for (Request* r : std::vector<Request*>(resident)) {
            if (r->inflight > 0 || r->state != Q_RESIDENT) continue;
            const int64_t left = r->nsteps - r->done_steps;
            if (left <= 0) {
                finish(r, MMVM_OK);
                continue;
            }
            const int64_t c = left < kChunkSteps ? left : kChunkSteps;
            const DevTables* T = nullptr;
            mmvm_status s = device_tables(r->order, &T);
            hipStream_t st = streams[r->stream];
            if (r->done_steps == 0 && r->stats.t_start == 0.0) r->stats.t_start = now();
            if (s == MMVM_OK)
                s = run_steps(*T, *r->ws, r->t0 + (double)r->done_steps * r->dt, r->dt, c, r->dx, r->dmom,
                              r->prec, st);
            if (s == MMVM_OK && hipEventRecord(r->ev, st) != hipSuccess) s = MMVM_EDEVICE;
            if (s != MMVM_OK) {
                finish(r, s);
                continue;
            }
            r->inflight = c;
        }
        // collect finished chunks
        bool progressed = false;
        for (Request* r : std::vector<Request*>(resident)) {
            if (r->inflight == 0) continue;
            hipError_t q = hipEventQuery(r->ev);
            if (q == hipErrorNotReady) continue;
            progressed = true;
            if (q != hipSuccess) {
                finish(r, MMVM_EDEVICE);
                continue;
            }
            r->done_steps += r->inflight;
            r->inflight = 0;
            // device-side checks of this request (its workspace is private)
            int f = 0;
            if (hipMemcpy(&f, r->ws->flag_ptr, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess) {
                finish(r, MMVM_EDEVICE);
                continue;
            }
            if (f & 2) finish(r, MMVM_ENONFINITE);
            else if (f & 1) finish(r, MMVM_EZEROCIRC);
            else if (r->done_steps >= r->nsteps) finish(r, MMVM_OK);
        }
        if (!progressed) {
            // let the device work; submissions wake us early
            cv_work.wait_for(lk, std::chrono::microseconds(200));
        }
    }
    cv_idle.notify_all();
}

extern "C" {

mmvm_status mmvm_server_create(size_t hbm_budget_bytes, int32_t max_slots, mmvm_server** out)
{
    if (!out || hbm_budget_bytes == 0 || max_slots < 1) return MMVM_EINVAL;
    *out = nullptr;
    std::unique_ptr<mmvm_server> s(new mmvm_server());
    s->budget = hbm_budget_bytes;
    s->max_slots = max_slots;
    s->t_origin = std::chrono::steady_clock::now();
    if (hipGetDevice(&s->device) != hipSuccess) return MMVM_EDEVICE;
    for (int i = 0; i < kStreams; ++i)
        if (hipStreamCreateWithFlags(&s->streams[i], hipStreamNonBlocking) != hipSuccess) return MMVM_EDEVICE;
    mmvm_server* raw = s.release();
    raw->worker = std::thread([raw] { raw->run(); });
    *out = raw;
    return MMVM_OK;
}

mmvm_status mmvm_submit(mmvm_server* srv, const mmvm_problem* prob, double t0, double dt, int64_t nsteps,
                        const double* x0, const double* mom0, mmvm_precision prec, uint64_t* ticket)
{
    if (!srv || !ticket || !x0 || !mom0) return MMVM_EINVAL;
    mmvm_status s = validate(prob);
    if (s != MMVM_OK) return s;
    if (nsteps < 0 || !std::isfinite(t0) || !std::isfinite(dt) || (prec != MMVM_FP64 && prec != MMVM_MIXED))
        return MMVM_EINVAL;
    const int n = prob->n, M = prob->order;
    const size_t K = (size_t)(M + 1) * (M + 2) / 2;
    for (int j = 0; j < n; ++j) {
        if (!std::isfinite(x0[2 * j]) || !std::isfinite(x0[2 * j + 1])) return MMVM_ENONFINITE;
        for (size_t k = 0; k < K; ++k)
            if (!std::isfinite(mom0[j * K + k])) return MMVM_ENONFINITE;
        if (n > 1 && mom0[j * K] == 0.0) return MMVM_EZEROCIRC;  // eq:mass
    }
    std::unique_ptr<Request> r(new Request());
    r->n = n;
    r->order = M;
    r->nu = prob->nu;
    r->t0 = t0;
    r->dt = dt;
    r->nsteps = nsteps;
    r->prec = prec;
    r->lambda0.assign(prob->lambda0, prob->lambda0 + n);
    r->x.assign(x0, x0 + 2 * (size_t)n);
    r->mom.assign(mom0, mom0 + (size_t)n * K);
    r->footprint = state_bytes(n, M) + Workspace::bytes_for(n, M, use_dd(M, prec), n == 1);
    if (r->footprint > srv->budget) return MMVM_EBUDGET;
    std::lock_guard<std::mutex> lk(srv->mu);
    if (srv->stop) return MMVM_EINVAL;
    r->ticket = srv->next_ticket++;
    r->stats.t_arrive = srv->now();
    *ticket = r->ticket;
    srv->queue.push_back(r.get());
    srv->all[r->ticket] = std::move(r);
    srv->cv_work.notify_one();
    return MMVM_OK;
}

mmvm_status mmvm_poll(mmvm_server* srv, uint64_t ticket, double* x_out, double* mom_out, mmvm_stats* stats)
{
    if (!srv) return MMVM_EINVAL;
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->all.find(ticket);
    if (it == srv->all.end()) return MMVM_ENOTFOUND;
    Request* r = it->second.get();
    if (r->state == Q_QUEUED || r->state == Q_RESIDENT) return MMVM_PENDING;
    mmvm_status st = r->status;
    if (st == MMVM_OK) {
        if (x_out) std::memcpy(x_out, r->x.data(), sizeof(double) * r->x.size());
        if (mom_out) std::memcpy(mom_out, r->mom.data(), sizeof(double) * r->mom.size());
    }
    if (stats) *stats = r->stats;
    srv->all.erase(it);
    return st;
}

mmvm_status mmvm_server_drain(mmvm_server* srv)
{
    if (!srv) return MMVM_EINVAL;
    std::unique_lock<std::mutex> lk(srv->mu);
    srv->cv_work.notify_one();
    srv->cv_idle.wait(lk, [srv] { return srv->queue.empty() && srv->resident.empty(); });
    return MMVM_OK;
}

mmvm_status mmvm_server_destroy(mmvm_server* srv)
{
    if (!srv) return MMVM_EINVAL;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stop = true;
        srv->cv_work.notify_all();
    }
    if (srv->worker.joinable()) srv->worker.join();
    for (int i = 0; i < kStreams; ++i)
        if (srv->streams[i]) (void)hipStreamDestroy(srv->streams[i]);
    delete srv;
    return MMVM_OK;
}

}  // extern "C"
