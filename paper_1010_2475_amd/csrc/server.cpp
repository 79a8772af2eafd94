// Continuous-batching solve server (mmvm_server_* in include/mmvm.h).
//
// A worker thread owns the device side.  Requests wait in arrival order until
// a slot is free and their HBM footprint (state + workspace) fits the budget;
// a request that does not fit lets later ones pass, for a bounded number of
// admissions, after which it is admitted before anything else (no
// starvation).  Admitted requests get a pooled slot (workspace, state buffer,
// pinned host words and an event, all reused by later requests; device memory
// is only grown, never freed before the server is destroyed), and join the
// resident set.  Every scheduling round the worker gives each idle resident
// request a chunk of RK4 steps on one of several HIP streams, so the kernels of
// different requests overlap on the device.  Single-vortex requests of one
// order, precision and step size are stepped together as one batch of
// independent solves (one launch of each kernel for the group), each member
// at its own time.  After a chunk, its error flags and, at the end, its state
// come back by asynchronous copies into pinned memory behind an event; the
// worker never waits on the device and never holds the lock during a device
// call.  Every request's arithmetic is that of stepping it alone, in the same
// chunks, so its result does not depend on what else is resident (bitwise).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstdlib>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <tuple>
#include <vector>

#include "api_internal.hpp"

namespace mmvm {
namespace {

constexpr int kStreams = 4;          // default streams: HIP's default hardware queues per process
constexpr int kMaxStreams = 16;       // MMVM_SERVER_STREAMS may ask for up to this many
constexpr int64_t kChunkSteps = 25;  // RK4 steps per scheduling quantum
constexpr int kMaxBypass = 64;       // admissions that may pass a waiting head

enum ReqState { Q_QUEUED, Q_RESIDENT, Q_DONE, Q_FAILED };

size_t state_doubles(int n, int M) { return (size_t)n * (2 + (size_t)(M + 1) * (M + 2) / 2); }

// Pooled device memory of one resident request (or of one batch group).
struct Slot {
    std::unique_ptr<Workspace> ws;
    double* state = nullptr;  // device: x [n][2], then mom [n][K]
    size_t state_cap = 0;     // doubles
    double* host = nullptr;   // pinned: the state coming back
    size_t host_cap = 0;
    int* hflag = nullptr;     // pinned: the workspace error flag after the last chunk
    hipEvent_t ev = nullptr;
    bool busy = false;
    ~Slot()
    {
        ws.reset();
        if (state) (void)hipFree(state);
        if (host) (void)hipHostFree(host);
        if (hflag) (void)hipHostFree(hflag);
        if (ev) (void)hipEventDestroy(ev);
    }
    mmvm_status reserve(size_t dev_doubles, size_t host_doubles)
    {
        if (!ws) ws.reset(new Workspace());
        if (!ev && hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) return MMVM_EDEVICE;
        if (!hflag && hipHostMalloc((void**)&hflag, sizeof(int) * 4, hipHostMallocDefault) != hipSuccess)
            return MMVM_ENOMEM;
        if (dev_doubles > state_cap) {
            if (state) (void)hipFree(state);
            state = nullptr;
            state_cap = 0;
            if (hipMalloc((void**)&state, sizeof(double) * dev_doubles) != hipSuccess) return MMVM_ENOMEM;
            state_cap = dev_doubles;
        }
        if (host_doubles > host_cap) {
            if (host) (void)hipHostFree(host);
            host = nullptr;
            host_cap = 0;
            if (hipHostMalloc((void**)&host, sizeof(double) * host_doubles, hipHostMallocDefault) != hipSuccess)
                return MMVM_ENOMEM;
            host_cap = host_doubles;
        }
        return MMVM_OK;
    }
};

struct Request {
    uint64_t ticket = 0;
    int n = 0, order = 0;
    double nu = 0.0, t0 = 0.0, dt = 0.0;
    int64_t nsteps = 0;
    mmvm_precision prec = MMVM_MIXED;
    std::vector<double> lambda0, x, mom;  // host input, then host result
    size_t footprint = 0;
    ReqState state = Q_QUEUED;
    mmvm_status status = MMVM_OK;
    mmvm_stats stats{};
    // worker-only fields
    int64_t done_steps = 0, inflight = 0;
    int stream = 0;
    Slot* slot = nullptr;
    bool batchable = false;  // a single vortex: may share launches with others of its key
    bool fetching = false;   // the final state is on its way back
};

// key of the single-vortex batches: order, precision, step size
typedef std::tuple<int, int, double> GroupKey;

// A chunk in flight for a batch group: its members, each at its own time.
struct GroupRun {
    GroupKey key;
    std::vector<Request*> members;
    Slot* slot = nullptr;
    int64_t steps = 0;
    int stream = 0;
};

}  // namespace
}  // namespace mmvm

using namespace mmvm;

struct mmvm_server {
    size_t budget = 0;
    int max_slots = 0;
    int device = 0;
    std::chrono::steady_clock::time_point t_origin;
    hipStream_t streams[kMaxStreams] = {};
    int nstreams = kStreams;

    std::mutex mu;                    // guards the fields below up to `stop`
    std::condition_variable cv_work;  // worker wake-up
    std::condition_variable cv_idle;  // drain
    std::deque<Request*> queue;
    std::vector<Request*> resident;
    std::map<uint64_t, std::unique_ptr<Request>> all;
    size_t used = 0;
    uint64_t next_ticket = 1;
    int head_bypassed = 0;
    bool stop = false;
    std::thread worker;

    // worker-only state
    std::vector<std::unique_ptr<Slot>> pool;
    std::vector<GroupRun> group_runs;
    int next_stream = 0;

    double now() const
    {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t_origin).count();
    }
    void run();
    void admit_locked(std::vector<Request*>& admitted);
    Slot* acquire_slot(size_t dev_doubles, size_t host_doubles, mmvm_status* s);
    mmvm_status start_request(Request* r);
    mmvm_status launch_chunk(Request* r);
    mmvm_status launch_group(GroupRun& g);
    mmvm_status fetch_result(Request* r);
    void complete_locked(Request* r, mmvm_status st);
};

void mmvm_server::admit_locked(std::vector<Request*>& admitted)
{
    // arrival order; a head that does not fit may be passed kMaxBypass times
    for (auto it = queue.begin(); it != queue.end();) {
        Request* r = *it;
        const bool is_head = it == queue.begin();
        if ((int)resident.size() >= max_slots) break;
        if (used + r->footprint <= budget) {
            used += r->footprint;
            r->state = Q_RESIDENT;
            r->stats.t_admit = now();
            resident.push_back(r);
            admitted.push_back(r);
            if (!is_head) ++head_bypassed;
            else head_bypassed = 0;
            it = queue.erase(it);
            continue;
        }
        if (head_bypassed >= kMaxBypass) break;  // the head waits for room, nobody passes it
        ++it;
    }
}

Slot* mmvm_server::acquire_slot(size_t dev_doubles, size_t host_doubles, mmvm_status* s)
{
    Slot* best = nullptr;
    for (auto& p : pool)  // a free slot that needs no growth, else any free slot
        if (!p->busy && (!best || (p->state_cap >= dev_doubles && best->state_cap < dev_doubles))) best = p.get();
    if (!best) {
        pool.emplace_back(new Slot());
        best = pool.back().get();
    }
    *s = best->reserve(dev_doubles, host_doubles);
    if (*s != MMVM_OK) return nullptr;
    best->busy = true;
    return best;
}

// device side of an admitted request: its slot, state upload, parameters
mmvm_status mmvm_server::start_request(Request* r)
{
    r->stream = next_stream;
    next_stream = (next_stream + 1) % nstreams;
    mmvm_status s = MMVM_OK;
    const size_t nd = state_doubles(r->n, r->order);
    r->slot = acquire_slot(nd, nd, &s);
    if (!r->slot) return s;
    hipStream_t st = streams[r->stream];
    Slot& sl = *r->slot;
    if (hipMemcpyAsync(sl.state, r->x.data(), sizeof(double) * 2 * r->n, hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemcpyAsync(sl.state + 2 * (size_t)r->n, r->mom.data(), sizeof(double) * r->mom.size(),
                       hipMemcpyHostToDevice, st) != hipSuccess)
        return MMVM_EDEVICE;
    if (!r->batchable) {
        if ((s = sl.ws->ensure(r->n, r->order, use_dd(r->order, r->prec), r->n == 1, st)) != MMVM_OK) return s;
        if ((s = sl.ws->set_params(r->lambda0.data(), nullptr, r->nu, r->n, st)) != MMVM_OK) return s;
        // a pooled workspace keeps the previous request's flag
        if (hipMemsetAsync(sl.ws->flag_ptr, 0, sizeof(int), st) != hipSuccess) return MMVM_EDEVICE;
    }
    // a batch group on another stream gathers this state after the upload's event
    if (hipEventRecord(sl.ev, st) != hipSuccess) return MMVM_EDEVICE;
    return MMVM_OK;
}

// one chunk of a request stepped on its own (multi-vortex, or a lone single)
mmvm_status mmvm_server::launch_chunk(Request* r)
{
    const int64_t left = r->nsteps - r->done_steps;
    const int64_t c = left < kChunkSteps ? left : kChunkSteps;
    const DevTables* T = nullptr;
    mmvm_status s = device_tables(r->order, &T);
    if (s != MMVM_OK) return s;
    hipStream_t st = streams[r->stream];
    Slot& sl = *r->slot;
    double* dx = sl.state;
    double* dm = sl.state + 2 * (size_t)r->n;
    s = run_steps(*T, *sl.ws, r->t0 + (double)r->done_steps * r->dt, r->dt, c, dx, dm, r->prec, st);
    if (s != MMVM_OK) return s;
    if (hipMemcpyAsync(sl.hflag, sl.ws->flag_ptr, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipEventRecord(sl.ev, st) != hipSuccess)
        return MMVM_EDEVICE;
    r->inflight = c;
    return MMVM_OK;
}

// one chunk of a group of single-vortex requests: their states are gathered
// into the group slot, stepped as one batch (member j at its own time), and
// scattered back; every member takes the same chunk length
mmvm_status mmvm_server::launch_group(GroupRun& g)
{
    const int nb = (int)g.members.size();
    const int M = std::get<0>(g.key);
    const mmvm_precision prec = (mmvm_precision)std::get<1>(g.key);
    const double dt = std::get<2>(g.key);
    const size_t K = (size_t)(M + 1) * (M + 2) / 2;
    const DevTables* T = nullptr;
    mmvm_status s = device_tables(M, &T);
    if (s != MMVM_OK) return s;
    hipStream_t st = streams[g.stream];
    Slot& sl = *g.slot;
    std::vector<double> lam(nb), nu(nb), toff(nb);
    for (int i = 0; i < nb; ++i) {
        Request* r = g.members[i];
        lam[i] = r->lambda0[0];
        nu[i] = r->nu;
        toff[i] = r->t0 + (double)r->done_steps * r->dt;  // the member's chunk start, as stepping it alone
        // the members' states (x then mom) live in their own slots; their last work on
        // another stream (the upload) is waited for through the slot's event
        if (hipStreamWaitEvent(st, r->slot->ev, 0) != hipSuccess) return MMVM_EDEVICE;
        if (hipMemcpyAsync(sl.state + 2 * (size_t)i, r->slot->state, sizeof(double) * 2, hipMemcpyDeviceToDevice,
                           st) != hipSuccess ||
            hipMemcpyAsync(sl.state + 2 * (size_t)nb + i * K, r->slot->state + 2, sizeof(double) * K,
                           hipMemcpyDeviceToDevice, st) != hipSuccess)
            return MMVM_EDEVICE;
    }
    if ((s = sl.ws->ensure(nb, M, use_dd(M, prec), true, st)) != MMVM_OK) return s;
    if ((s = sl.ws->set_params(lam.data(), nu.data(), 0.0, nb, st, toff.data())) != MMVM_OK) return s;
    if (hipMemsetAsync(sl.ws->flag_ptr, 0, sizeof(int), st) != hipSuccess) return MMVM_EDEVICE;
    s = run_steps(*T, *sl.ws, 0.0, dt, g.steps, sl.state, sl.state + 2 * (size_t)nb, prec, st);
    if (s != MMVM_OK) return s;
    for (int i = 0; i < nb; ++i) {
        Request* r = g.members[i];
        if (hipMemcpyAsync(r->slot->state + 2, sl.state + 2 * (size_t)nb + i * K, sizeof(double) * K,
                           hipMemcpyDeviceToDevice, st) != hipSuccess)
            return MMVM_EDEVICE;
    }
    if (hipMemcpyAsync(sl.hflag, sl.ws->flag_ptr, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipEventRecord(sl.ev, st) != hipSuccess)
        return MMVM_EDEVICE;
    for (Request* r : g.members) r->inflight = g.steps;
    return MMVM_OK;
}

// the final state into the slot's pinned buffer, behind the slot's event
mmvm_status mmvm_server::fetch_result(Request* r)
{
    hipStream_t st = streams[r->stream];
    Slot& sl = *r->slot;
    const size_t nd = state_doubles(r->n, r->order);
    if (hipMemcpyAsync(sl.host, sl.state, sizeof(double) * nd, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipEventRecord(sl.ev, st) != hipSuccess)
        return MMVM_EDEVICE;
    r->fetching = true;
    return MMVM_OK;
}

// caller holds mu; the request's device work has completed
void mmvm_server::complete_locked(Request* r, mmvm_status st)
{
    if (st == MMVM_OK && r->slot) {
        const double* h = r->slot->host;
        std::memcpy(r->x.data(), h, sizeof(double) * 2 * r->n);
        std::memcpy(r->mom.data(), h + 2 * (size_t)r->n, sizeof(double) * r->mom.size());
    }
    if (r->slot) r->slot->busy = false;
    r->slot = nullptr;
    used -= r->footprint;
    r->state = st == MMVM_OK ? Q_DONE : Q_FAILED;
    r->status = st;
    r->stats.t_done = now();
    r->stats.steps = r->done_steps;
    resident.erase(std::find(resident.begin(), resident.end(), r));
}

void mmvm_server::run()
{
    (void)hipSetDevice(device);
    std::vector<Request*> admitted, idle, inflight;
    std::vector<std::pair<Request*, mmvm_status>> ended;
    std::unique_lock<std::mutex> lk(mu);
    while (true) {
        admitted.clear();
        admit_locked(admitted);
        if (stop && queue.empty() && resident.empty()) break;
        if (resident.empty()) {
            cv_idle.notify_all();
            if (stop) break;
            cv_work.wait(lk);
            continue;
        }
        for (Request* r : admitted)
            if (r->stats.t_start == 0.0) r->stats.t_start = now();
        std::vector<Request*> snapshot(resident);
        lk.unlock();

        // ---- device work, without the lock
        ended.clear();
        for (Request* r : admitted) {
            r->batchable = r->n == 1;
            const mmvm_status s = start_request(r);
            if (s != MMVM_OK) ended.push_back(std::make_pair(r, s));
        }
        // completions: chunks whose event fired (groups first: their members share one event)
        bool progressed = false;
        for (size_t gi = 0; gi < group_runs.size();) {
            GroupRun& g = group_runs[gi];
            const hipError_t q = hipEventQuery(g.slot->ev);
            if (q == hipErrorNotReady) {
                ++gi;
                continue;
            }
            progressed = true;
            const int f = q == hipSuccess ? *g.slot->hflag : 0;
            for (Request* r : g.members) {
                r->inflight = 0;
                if (q != hipSuccess) {
                    ended.push_back(std::make_pair(r, MMVM_EDEVICE));
                    continue;
                }
                r->done_steps += g.steps;
            }
            if (q == hipSuccess && (f & 2)) {
                // some member turned non-finite: the group's flag cannot say which, so every
                // member leaves the batch and is stepped alone from now on (its state is kept)
                for (Request* r : g.members) r->batchable = false;
            }
            g.slot->busy = false;
            group_runs.erase(group_runs.begin() + (long)gi);
        }
        for (Request* r : snapshot) {
            if (!r->slot) continue;
            if (!r->fetching && (r->inflight == 0 || r->batchable)) continue;  // group chunks complete above
            const hipError_t q = hipEventQuery(r->slot->ev);
            if (q == hipErrorNotReady) continue;
            progressed = true;
            if (q != hipSuccess) {
                ended.push_back(std::make_pair(r, MMVM_EDEVICE));
                continue;
            }
            if (r->fetching) {  // the final state is in the slot's pinned buffer
                ended.push_back(std::make_pair(r, MMVM_OK));
                continue;
            }
            r->done_steps += r->inflight;
            r->inflight = 0;
            const int f = *r->slot->hflag;  // device-side checks of this request's workspace
            if (f & 2) ended.push_back(std::make_pair(r, MMVM_ENONFINITE));
            else if (f & 1) ended.push_back(std::make_pair(r, MMVM_EZEROCIRC));
        }
        // batched members that left a group after a non-finite flag need their own workspace
        for (Request* r : snapshot)
            if (r->slot && !r->batchable && r->n == 1 && r->inflight == 0 && !r->fetching && r->slot->ws &&
                r->slot->ws->N != 1) {
                hipStream_t st = streams[r->stream];
                mmvm_status s = r->slot->ws->ensure(1, r->order, use_dd(r->order, r->prec), true, st);
                if (s == MMVM_OK) s = r->slot->ws->set_params(r->lambda0.data(), nullptr, r->nu, 1, st);
                if (s == MMVM_OK && hipMemsetAsync(r->slot->ws->flag_ptr, 0, sizeof(int), st) != hipSuccess)
                    s = MMVM_EDEVICE;
                if (s != MMVM_OK) ended.push_back(std::make_pair(r, s));
            }
        // new chunks: batchable singles grouped by (order, precision, dt), the rest alone
        std::map<GroupKey, std::vector<Request*>> groups;
        for (Request* r : snapshot) {
            if (!r->slot || r->inflight > 0 || r->fetching) continue;
            bool gone = false;
            for (auto& e : ended) gone |= e.first == r;
            if (gone) continue;
            if (r->done_steps >= r->nsteps) {
                const mmvm_status s = fetch_result(r);
                if (s != MMVM_OK) ended.push_back(std::make_pair(r, s));
                continue;
            }
            if (r->batchable) {
                groups[std::make_tuple(r->order, (int)r->prec, r->dt)].push_back(r);
                continue;
            }
            const mmvm_status s = launch_chunk(r);
            if (s != MMVM_OK) ended.push_back(std::make_pair(r, s));
        }
        for (auto& kv : groups) {
            // members advance in equal chunks: the shortest remainder sets the chunk, so
            // a member's chunk sequence is that of stepping it alone (25 steps, then the rest)
            std::vector<Request*>& ms = kv.second;
            std::vector<Request*> full, tail;
            for (Request* r : ms) (r->nsteps - r->done_steps >= kChunkSteps ? full : tail).push_back(r);
            for (int pass = 0; pass < 2; ++pass) {
                std::vector<Request*>& part = pass == 0 ? full : tail;
                // members with a shorter remainder each take their own (exact) last chunk
                std::map<int64_t, std::vector<Request*>> by_len;
                for (Request* r : part) {
                    const int64_t left = r->nsteps - r->done_steps;
                    by_len[left < kChunkSteps ? left : kChunkSteps].push_back(r);
                }
                for (auto& bl : by_len) {
                    GroupRun g;
                    g.key = kv.first;
                    g.members = bl.second;
                    g.steps = bl.first;
                    g.stream = next_stream;
                    next_stream = (next_stream + 1) % nstreams;
                    mmvm_status s = MMVM_OK;
                    const size_t nd = state_doubles((int)g.members.size(), std::get<0>(g.key));
                    g.slot = acquire_slot(nd, 0, &s);
                    if (g.slot) s = launch_group(g);
                    if (s != MMVM_OK) {
                        if (g.slot) g.slot->busy = false;
                        for (Request* r : g.members) ended.push_back(std::make_pair(r, s));
                        continue;
                    }
                    group_runs.push_back(std::move(g));
                }
            }
        }
        lk.lock();
        for (auto& e : ended) {
            Request* r = e.first;
            if (r->state != Q_RESIDENT) continue;
            complete_locked(r, e.second);
            progressed = true;
        }
        if (!progressed && admitted.empty()) cv_work.wait_for(lk, std::chrono::microseconds(100));
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
    if (const char* e = std::getenv("MMVM_SERVER_STREAMS")) {
        const int n = std::atoi(e);
        if (n >= 1 && n <= kMaxStreams) s->nstreams = n;
    }
    for (int i = 0; i < s->nstreams; ++i)
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
    // state + the request's own workspace (a single vortex may also run alone)
    r->footprint = sizeof(double) * state_doubles(n, M) + Workspace::bytes_for(n, M, use_dd(M, prec), n == 1);
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
    for (int i = 0; i < kMaxStreams; ++i)
        if (srv->streams[i]) (void)hipStreamSynchronize(srv->streams[i]);
    srv->pool.clear();
    for (int i = 0; i < kMaxStreams; ++i)
        if (srv->streams[i]) (void)hipStreamDestroy(srv->streams[i]);
    delete srv;
    return MMVM_OK;
}

}  // extern "C"
