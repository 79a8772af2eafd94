// C ABI of libmmvm (declarations and contracts in include/mmvm.h).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <algorithm>
#include <map>
#include <memory>
#include <mutex>
#include <vector>

#include "../../include/mmvm.h"
#include "api_internal.hpp"
#include "kernels.hpp"
#include "tables.hpp"

namespace mmvm {

// ---------------------------------------------------------------------------
// device tables (per device, per order)
// ---------------------------------------------------------------------------
namespace {

struct DevTablesOwner {
    DevTables t;
    std::vector<void*> bufs;
    ~DevTablesOwner()
    {
        for (void* p : bufs) (void)hipFree(p);
    }
};

std::mutex g_tab_mu;
std::map<std::pair<int, int>, std::unique_ptr<DevTablesOwner>> g_dev_tables;

// Tables are copied on a stream of their own and waited for there: a
// device-wide synchronisation would stall behind every solve in flight (the
// first request of a new order arrives while others run).
std::map<int, hipStream_t> g_upload_streams;  // per device, under g_tab_mu

template <typename V>
const typename V::value_type* upload(DevTablesOwner& o, const V& v, hipStream_t us, hipError_t& err)
{
    typedef typename V::value_type E;
    if (err != hipSuccess) return nullptr;
    void* p = nullptr;
    size_t n = v.size() * sizeof(E);
    if (n == 0) n = sizeof(E);
    err = hipMalloc(&p, n);
    if (err != hipSuccess) return nullptr;
    o.bufs.push_back(p);
    if (!v.empty()) {
        err = hipMemcpyAsync(p, v.data(), v.size() * sizeof(E), hipMemcpyHostToDevice, us);
        if (err == hipSuccess) err = hipStreamSynchronize(us);  // v may be a temporary
    }
    return (const E*)p;
}

// Task lists of the double-double stage 2, one per workgroup (k2, pass, row
// parity): steps A and C visit their (row, l2) and (k1, l1-slot) sums in
// decreasing order of length, so the lanes of a wavefront run loops of about
// equal trip count.  Entries (hi << 8 | lo), padded with -1.
void dd_task_lists(int M, std::vector<int32_t>& la, std::vector<int32_t>& lc)
{
    const int M1 = M + 1, GM = 2 * M, H = (M1 + 1) >> 1;
    la.assign((size_t)M1 * 4 * M1 * M1, -1);
    lc.assign((size_t)M1 * 4 * M1 * H, -1);
    std::vector<std::pair<int, int32_t>> v;
    for (int k2 = 0; k2 <= M; ++k2)
        for (int pass = 0; pass < 2; ++pass)
            for (int par = 0; par < 2; ++par) {
                const size_t b = ((size_t)k2 * 2 + pass) * 2 + par;
                const int nrp = (2 * M - par) / 2 + 1, off = pass == 0 ? 1 : -1;
                v.clear();
                for (int l2 = 0; l2 <= M; ++l2)
                    for (int r = 0; r < nrp; ++r) {
                        const int g1 = par + 2 * r;
                        const int imax = pass == 0 ? std::min(l2, k2) : std::min(l2, k2 - 1);
                        const int over = k2 + l2 + off + g1 - GM;
                        const int ilo = over > 0 ? (over + 1) >> 1 : 0;
                        v.push_back(std::make_pair(std::max(0, imax - ilo + 1), (int32_t)((r << 8) | l2)));
                    }
                std::stable_sort(v.begin(), v.end(), [](const std::pair<int, int32_t>& a,
                                                        const std::pair<int, int32_t>& c) { return a.first > c.first; });
                for (size_t t = 0; t < v.size(); ++t) la[b * M1 * M1 + t] = v[t].second;
                v.clear();
                for (int k1 = 0; k1 <= M - k2; ++k1)
                    for (int q = 0; q < H; ++q) {
                        const int l1 = 2 * q + ((par + k1 + 1) & 1);
                        int trip = 0;
                        if (l1 <= M) {
                            if (pass == 0) trip = std::min(l1, k1 - 1) + 1;
                            else trip = std::min(l1, k1) + 1 - (k1 + l1 + 1 > GM ? 1 : 0);
                        }
                        v.push_back(std::make_pair(std::max(0, trip), (int32_t)((k1 << 8) | q)));
                    }
                std::stable_sort(v.begin(), v.end(), [](const std::pair<int, int32_t>& a,
                                                        const std::pair<int, int32_t>& c) { return a.first > c.first; });
                for (size_t t = 0; t < v.size(); ++t) lc[b * M1 * H + t] = v[t].second;
            }
}

}  // namespace

const DevTables* find_device_tables(int M)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return nullptr;
    std::lock_guard<std::mutex> lk(g_tab_mu);
    auto it = g_dev_tables.find(std::make_pair(dev, M));
    return it == g_dev_tables.end() ? nullptr : &it->second->t;
}

mmvm_status device_tables(int M, const DevTables** out)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return MMVM_EDEVICE;
    std::lock_guard<std::mutex> lk(g_tab_mu);
    auto key = std::make_pair(dev, M);
    auto it = g_dev_tables.find(key);
    if (it != g_dev_tables.end()) {
        *out = &it->second->t;
        return MMVM_OK;
    }
    const Tables& H = get_tables(M);
    std::unique_ptr<DevTablesOwner> o(new DevTablesOwner());
    hipError_t err = hipSuccess;
    hipStream_t& us = g_upload_streams[dev];
    if (!us && (err = hipStreamCreateWithFlags(&us, hipStreamNonBlocking)) != hipSuccess) {
        us = nullptr;
        report_hip_error(err, "table upload stream");
        return MMVM_EDEVICE;
    }
    DevTables& d = o->t;
    d.M = H.M; d.K = H.K; d.P = H.P; d.GM = H.GM; d.KG = H.KG; d.T0N = H.T0N;
    d.t0_hi = upload(*o, H.t0_hi, us, err);
    d.t0_lo = upload(*o, H.t0_lo, us, err);
    d.f0_hi = upload(*o, H.f0_hi, us, err);
    d.f0_lo = upload(*o, H.f0_lo, us, err);
    d.f1_hi = upload(*o, H.f1_hi, us, err);
    d.f1_lo = upload(*o, H.f1_lo, us, err);
    d.binom = upload(*o, H.binom, us, err);
    d.fd0 = upload(*o, H.fd0, us, err);
    d.fd1 = upload(*o, H.fd1, us, err);
    d.fd0_lo = upload(*o, H.fd0_lo, us, err);
    d.fd1_lo = upload(*o, H.fd1_lo, us, err);
    {
        std::vector<int32_t> la, lc;
        if (M > kDDThreshold && M <= MMVM_MAX_ORDER) dd_task_lists(M, la, lc);
        d.dd_la = upload(*o, la, us, err);
        d.dd_lc = upload(*o, lc, us, err);
    }
    {
        // zero-padded operands of the matrix-core stage 2 (see S2Shape)
        std::vector<double> wpad, cpad;
        if (mfma_order(M)) {
            const S2Shape sh(M, 0);
            const int M1 = M + 1, KA = sh.KA, LP = sh.LP;
            wpad.assign((size_t)M1 * 2 * KA * LP, 0.0);
            for (int k2 = 0; k2 <= M; ++k2)
                for (int pass = 0; pass < 2; ++pass) {
                    const std::vector<double>& F = pass == 0 ? H.f0_hi : H.f1_hi;
                    const int off2 = pass == 0 ? 1 : -1, imaxk = pass == 0 ? k2 : k2 - 1;
                    double* w = wpad.data() + ((size_t)k2 * 2 + pass) * KA * LP;
                    for (int l2 = 0; l2 <= M; ++l2)
                        for (int i = 0; i <= l2 && i <= imaxk; ++i) {
                            const int g2 = k2 + l2 + off2 - 2 * i;
                            if (g2 >= 0 && g2 < KA) w[(size_t)g2 * LP + l2] = F[((size_t)k2 * M1 + l2) * M1 + i];
                        }
                }
            cpad.assign((size_t)LP * LP, 0.0);
            for (int l = 0; l <= M; ++l)
                for (int i = 0; i <= l; ++i) cpad[(size_t)l * LP + i] = H.binom[(size_t)l * M1 + i];
        }
        d.wpad = upload(*o, wpad, us, err);
        d.cpad = upload(*o, cpad, us, err);
        std::vector<double> t0d;
        if (mfma_order(M)) {
            const T0Shape tz(M);
            t0d.assign((size_t)tz.T0R * tz.TP, 0.0);
            for (int a = 0; a <= H.T0N; ++a)
                for (int b = 0; a + b <= H.T0N; ++b) t0d[(size_t)a * tz.TP + b] = H.t0_hi[tri(a, b)];
        }
        d.t0d = upload(*o, t0d, us, err);
        std::vector<double> c1d;
        if (mfma_order(M)) {
            const int LP = S2Shape(M, 0).LP;
            c1d.assign((size_t)LP * LP, 0.0);
            for (int k1 = 0; k1 <= M; ++k1)
                for (int k2 = 0; k1 + k2 <= M; ++k2) c1d[(size_t)k1 * LP + k2] = H.c1_hi[tri(k1, k2)];
        }
        d.c1d = upload(*o, c1d, us, err);
    }
    d.c1_hi = upload(*o, H.c1_hi, us, err);
    d.c1_lo = upload(*o, H.c1_lo, us, err);
    d.kap0 = upload(*o, H.kap0, us, err);
    d.kap1 = upload(*o, H.kap1, us, err);
    d.hol = upload(*o, H.hol, us, err);
    std::vector<double> rcp(128, 0.0);
    for (int i = 1; i < 128; ++i) rcp[i] = 1.0 / (double)i;
    d.rcp = upload(*o, rcp, us, err);
    // every copy has completed (waited for on the upload stream), so kernels on
    // any stream may read the tables
    if (err != hipSuccess) {
        report_hip_error(err, "table upload");
        return err == hipErrorOutOfMemory ? MMVM_ENOMEM : MMVM_EDEVICE;
    }
    *out = &o->t;
    g_dev_tables[key] = std::move(o);
    return MMVM_OK;
}

// ---------------------------------------------------------------------------
// workspaces (per device and stream), grown on demand
// ---------------------------------------------------------------------------
void Workspace::drop_graph()
{
    if (graph) (void)hipGraphExecDestroy(graph);
    graph = nullptr;
    graph_kind = graph_M = graph_N = -1;
    for (auto& g : retired) {
        (void)hipGraphExecDestroy(g.first);
        (void)hipEventDestroy(g.second);
    }
    retired.clear();
}

void Workspace::retire_graph()
{
    for (size_t i = 0; i < retired.size();) {
        if (hipEventQuery(retired[i].second) == hipSuccess) {
            (void)hipGraphExecDestroy(retired[i].first);
            (void)hipEventDestroy(retired[i].second);
            retired.erase(retired.begin() + (long)i);
        } else {
            ++i;
        }
    }
    (void)hipGetLastError();
    if (!graph) return;
    // the event keeps the last replays' place; a fresh one serves the next graph
    retired.emplace_back(graph, graph_done);
    graph = nullptr;
    graph_done = nullptr;
    graph_kind = graph_M = graph_N = -1;
}

// callers synchronise the stream first (queued work may still use the buffer)
void Workspace::release()
{
    // the parameter upload reads par_cache until its event
    if (par_event) (void)hipEventSynchronize(par_event);
    drop_graph();
    if (base) (void)hipFree(base);
    base = nullptr;
    bytes = 0;
    clock = nullptr;
    par_cache.clear();
}

Workspace::~Workspace()
{
    release();
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    if (par_event) (void)hipEventDestroy(par_event);
    if (graph_done) (void)hipEventDestroy(graph_done);
}

namespace {
struct Layout {
    size_t flag, lam0, xs, ys, accx, accm, lam2[2], alpha[2], alphaT[2], alphaT32[2], alphaD[2], alphaS[2], sself,
        sselflo, spair, ppart, fmask, rank, perm, xsS, lam2S[2], chunkmp, spad, ystate[2], accd, gpartd, gpart, clock,
        total;
};
Layout layout_for(int N_, int M_, bool need_dd, bool solo)
{
    const int K = (M_ + 1) * (M_ + 2) / 2;
    const int GM = M_ == 0 ? 1 : 2 * M_;
    const int KG = (GM + 1) * (GM + 2) / 2;
    Layout L{};
    size_t need = 0;
    auto add = [&](size_t n) {
        size_t o = need;
        need += (n + 255) & ~(size_t)255;  // 256-byte aligned regions: whole cache lines
        return o;
    };
    L.flag = add(sizeof(int) * 16);  // first: fixed offset across layouts
    L.lam0 = add(sizeof(double) * 3 * N_);  // lambda_{j,0}^2, nu_j and the time offset of vortex j
    L.xs = add(sizeof(double) * 2 * N_);
    L.ys = add(sizeof(double) * (size_t)N_ * K);
    L.accx = add(sizeof(double) * 2 * N_);
    L.accm = add(sizeof(double) * (size_t)N_ * K);
    for (int b = 0; b < 2; ++b) {
        L.lam2[b] = add(sizeof(double) * N_);
        L.alpha[b] = add(sizeof(double) * (size_t)N_ * K);
        L.alphaT[b] = add(sizeof(double) * (size_t)N_ * K);
        L.alphaT32[b] = add(sizeof(float) * (size_t)N_ * K);
        const bool mx = stage2_uses_mfma(M_, false, solo);
        const S2Shape sh(M_, 0);
        L.alphaD[b] = add(mx ? sizeof(double) * (size_t)N_ * sh.LA() * sh.LP : 0);
        L.alphaS[b] = add(mx ? sizeof(double) * (size_t)N_ * sh.LP * sh.LP : 0);
    }
    L.sself = add(sizeof(double) * (size_t)N_ * KG);
    L.sselflo = add(need_dd ? sizeof(double) * (size_t)N_ * KG : 0);
    L.spair = add(sizeof(double) * (size_t)N_ * KG);
    // partial tables of the few-vortex pair kernel (interacting vortices of the unrolled orders)
    const bool split = !solo && N_ > 1 && M_ <= kMaxPairOrder && pair_split_groups(N_) > 1;
    L.ppart = add(split ? sizeof(double) * (size_t)N_ * pair_split_groups(N_) * KG : 0);
    // far-field chunk mask of the unrolled pair kernel
    const bool far = !solo && N_ > 1 && M_ <= kMaxPairOrder && N_ <= kPairFarMaxN;
    L.fmask = add(far ? (size_t)N_ * pair_mask_stride(N_) : 0);
    // the sources in spatial order
    const bool sorted = far && N_ >= kPairFarAlwaysN;
    L.rank = add(sorted ? sizeof(int) * N_ : 0);
    L.perm = add(sorted ? sizeof(int) * N_ : 0);
    L.xsS = add(sorted ? sizeof(double) * 2 * N_ : 0);
    for (int q = 0; q < 2; ++q) L.lam2S[q] = add(sorted ? sizeof(double) * N_ : 0);
    L.chunkmp = add(sorted ? sizeof(double) * (size_t)far_records(N_) * kChunkRec : 0);
    L.spad = add(stage2_uses_mfma(M_, false, solo) ? sizeof(double) * (size_t)N_ * S2Shape(M_, 0).spad() : 0);
    {
        const size_t dense = stage2_uses_mfma(M_, false, solo) ? sizeof(double) * (size_t)N_ * S2Shape(M_, 0).LP * S2Shape(M_, 0).LP : 0;
        for (int b = 0; b < 2; ++b) L.ystate[b] = add(dense);
        L.accd = add(dense);
        L.gpartd = add(4 * dense);
    }
    L.gpart = add(sizeof(double) * (size_t)N_ * 4 * K * 2);
    L.clock = add(sizeof(DevClock));
    L.total = need;
    return L;
}
}  // namespace

size_t stage_layout(char* b, int N_, int M_, bool need_dd, bool solo, StageBufs* out, DevClock** clock,
                    double** par)
{
    const Layout L = layout_for(N_, M_, need_dd, solo);
    if (!b) return L.total;
    StageBufs& bufs = *out;
    bufs = StageBufs{};
    bufs.N = N_;
    bufs.interact = (!solo && N_ > 1) ? 1 : 0;
    bufs.lam0sq = (const double*)(b + L.lam0);
    bufs.nuv = (const double*)(b + L.lam0) + N_;
    bufs.toff = (const double*)(b + L.lam0) + 2 * (size_t)N_;
    bufs.xs = (double*)(b + L.xs);
    bufs.ys = (double*)(b + L.ys);
    bufs.accx = (double*)(b + L.accx);
    bufs.accm = (double*)(b + L.accm);
    const bool mx = stage2_uses_mfma(M_, false, solo);
    for (int q = 0; q < 2; ++q) {
        bufs.lam2[q] = (double*)(b + L.lam2[q]);
        bufs.alpha[q] = (double*)(b + L.alpha[q]);
        bufs.alphaT[q] = (double*)(b + L.alphaT[q]);
        bufs.alphaT32[q] = (float*)(b + L.alphaT32[q]);
        bufs.alphaD[q] = mx ? (double*)(b + L.alphaD[q]) : nullptr;
        bufs.alphaS[q] = mx ? (double*)(b + L.alphaS[q]) : nullptr;
    }
    bufs.s_self = (double*)(b + L.sself);
    bufs.s_self_lo = need_dd ? (double*)(b + L.sselflo) : nullptr;
    bufs.s_pair = (double*)(b + L.spair);
    bufs.p_part = (!solo && N_ > 1 && M_ <= kMaxPairOrder && pair_split_groups(N_) > 1) ? (double*)(b + L.ppart)
                                                                                          : nullptr;
    bufs.pair_groups = 0;
    const bool far = !solo && N_ > 1 && M_ <= kMaxPairOrder && N_ <= kPairFarMaxN;
    bufs.far_mask = far ? (unsigned char*)(b + L.fmask) : nullptr;
    const bool sorted = far && N_ >= kPairFarAlwaysN;
    bufs.rank = sorted ? (const int*)(b + L.rank) : nullptr;
    bufs.perm = sorted ? (const int*)(b + L.perm) : nullptr;
    bufs.xsS = sorted ? (double*)(b + L.xsS) : bufs.xs;
    for (int q = 0; q < 2; ++q) bufs.lam2S[q] = sorted ? (double*)(b + L.lam2S[q]) : bufs.lam2[q];
    bufs.chunk_mp = sorted ? (double*)(b + L.chunkmp) : nullptr;
    bufs.s_pad = (double*)(b + L.spad);
    for (int q = 0; q < 2; ++q) bufs.ystate[q] = mx ? (double*)(b + L.ystate[q]) : nullptr;
    bufs.accD = mx ? (double*)(b + L.accd) : nullptr;
    bufs.gpartD = mx ? (double*)(b + L.gpartd) : nullptr;
    bufs.gpart = (double*)(b + L.gpart);
    bufs.flag = (int*)(b + L.flag);
    if (clock) *clock = (DevClock*)(b + L.clock);
    if (par) *par = (double*)(b + L.lam0);
    return L.total;
}

size_t Workspace::bytes_for(int N_, int M_, bool need_dd, bool solo)
{
    return stage_layout(nullptr, N_, M_, need_dd, solo, nullptr, nullptr, nullptr);
}

mmvm_status Workspace::ensure(int N_, int M_, bool need_dd, bool solo, hipStream_t st)
{
    const size_t need = bytes_for(N_, M_, need_dd, solo);
    if (need > bytes) {
        // the old buffer may still be used by queued work on this stream
        if (base) {
            if (hipStreamSynchronize(st) != hipSuccess) return MMVM_EDEVICE;
            // keep a latched error across the reallocation
            int f = 0;
            (void)hipMemcpy(&f, flag_ptr, sizeof(int), hipMemcpyDeviceToHost);
            latched |= f;
            release();
        }
        void* p = nullptr;
        hipError_t e = hipMalloc(&p, need);
        if (e != hipSuccess) {
            report_hip_error(e, "workspace hipMalloc");
            return e == hipErrorOutOfMemory ? MMVM_ENOMEM : MMVM_EDEVICE;
        }
        base = (char*)p;
        bytes = need;
        // zeroed on the workspace's stream (the error flag starts at 0): a plain
        // hipMemset runs on the null stream, which does not order work on
        // non-blocking streams
        if (hipMemsetAsync(base, 0, need, st) != hipSuccess) return MMVM_EDEVICE;
        par_cache.clear();
    }
    N = N_;
    M = M_;
    stage_layout(base, N_, M_, need_dd, solo, &bufs, &clock, &par_dev);
    flag_ptr = bufs.flag;
    return MMVM_OK;
}

mmvm_status Workspace::set_params(const double* lambda0, const double* nu, double nu0, int N_, hipStream_t st,
                                  const double* toff)
{
    std::vector<double> p(3 * (size_t)N_);
    for (int j = 0; j < N_; ++j) {
        p[j] = lambda0[j] * lambda0[j];
        p[N_ + j] = nu ? nu[j] : nu0;
        p[2 * (size_t)N_ + j] = toff ? toff[j] : 0.0;
    }
    if (p == par_cache) return MMVM_OK;
    // The device copy may be read by queued work, so the update is ordered on
    // the stream; its source is the cached host copy, which is replaced only
    // after the previous update has completed (its event, not the stream).
    if (par_event && hipEventSynchronize(par_event) != hipSuccess) return MMVM_EDEVICE;
    if (!par_event && hipEventCreateWithFlags(&par_event, hipEventDisableTiming) != hipSuccess) {
        par_event = nullptr;
        return MMVM_EDEVICE;
    }
    par_cache.swap(p);
    if (hipMemcpyAsync(par_dev, par_cache.data(), sizeof(double) * par_cache.size(), hipMemcpyHostToDevice, st) !=
            hipSuccess ||
        hipEventRecord(par_event, st) != hipSuccess) {
        par_cache.clear();
        return MMVM_EDEVICE;
    }
    return MMVM_OK;
}

namespace {
std::mutex g_ws_mu;
std::map<std::pair<int, hipStream_t>, std::unique_ptr<Workspace>> g_ws;
}  // namespace

Workspace* workspace_for(hipStream_t st)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return nullptr;
    std::lock_guard<std::mutex> lk(g_ws_mu);
    auto& w = g_ws[std::make_pair(dev, st)];
    if (!w) w.reset(new Workspace());
    return w.get();
}

mmvm_status validate(const mmvm_problem* prob)
{
    if (!prob) return MMVM_EINVAL;
    if (prob->n < 1 || prob->order < 0 || prob->order > MMVM_MAX_ORDER) return MMVM_EORDER;
    if (!(prob->nu >= 0.0) || !std::isfinite(prob->nu) || !prob->lambda0) return MMVM_EINVAL;
    for (int j = 0; j < prob->n; ++j)
        if (!(prob->lambda0[j] > 0.0) || !std::isfinite(prob->lambda0[j])) return MMVM_EINVAL;
    if (prob->n > 1 && !pair_order_supported(prob->order)) return MMVM_EORDER;
    return MMVM_OK;
}

bool use_dd(int M, mmvm_precision prec) { return prec == MMVM_FP64 && M > kDDThreshold; }

void report_hip_error(hipError_t e, const char* where)
{
    if (e == hipSuccess || std::getenv("MMVM_QUIET")) return;
    std::fprintf(stderr, "libmmvm: %s failed: %s\n", where, hipGetErrorString(e));
}

static mmvm_status hip_status(hipError_t e, const char* where)
{
    if (e == hipSuccess) return MMVM_OK;
    report_hip_error(e, where);
    return e == hipErrorOutOfMemory ? MMVM_ENOMEM : MMVM_EDEVICE;
}

// the kernels of one stage whose inputs are in buffer A.cur (prep already ran);
// shape: the pair kernel's launch shape, or null for the autotuner's
mmvm_status run_stage_bufs(const DevTables& T, const StageBufs& B, mmvm_precision prec, const StageArgs& A,
                           hipStream_t st, const PairShape* shape)
{
    const bool pair = B.interact != 0;
    const bool f32 = prec == MMVM_MIXED;
    const bool dd = use_dd(T.M, prec);
    hipError_t e;
    void* tk;
    if (!stage2_fuses_self(T.M, dd, !B.interact)) {
        tk = timing_begin(st);
        e = launch_self(T, B, A.cur, dd, st);
        timing_end(tk, "self", st);
        if (e != hipSuccess) return hip_status(e, "k_self launch");
    }
    StageBufs B2 = B;  // the stage-2 kernel learns how the pair table was left
    B2.pair_groups = 0;
    if (pair) {
        PairShape used;
        tk = timing_begin(st);
        if (shape) {
            used = *shape;
            e = launch_pair_shape(T, B, A.cur, f32, used, st);
        } else {
            e = launch_pair(T, B, A.cur, f32, st, &used);
        }
        timing_end(tk, "pair", st);
        if (e != hipSuccess) return hip_status(e, "k_pair launch");
        if (used.kind == 1 && T.M <= kMaxPairOrder && pair_split_groups(B.N) > 1) B2.pair_groups = pair_split_groups(B.N);
        if (dd || stage2_uses_mfma(T.M, dd, false)) {
            e = launch_pair_into_stage2(T, B, dd, st);
            if (e != hipSuccess) return hip_status(e, "k_pair_into_stage2 launch");
        }
    }
    tk = timing_begin(st);
    e = launch_stage2(T, B2, A, dd, st);
    timing_end(tk, "stage2", st);
    if (e != hipSuccess) return hip_status(e, "k_stage2 launch");
    if (!stage2_needs_emit(T.M, dd, !B.interact)) return MMVM_OK;
    tk = timing_begin(st);
    e = launch_emit(T, B, A, dd, st);
    timing_end(tk, "emit", st);
    return hip_status(e, "k_emit launch");
}

mmvm_status run_stage(const DevTables& T, Workspace& W, mmvm_precision prec, const StageArgs& A, hipStream_t st)
{
    return run_stage_bufs(T, W.bufs, prec, A, st, nullptr);
}

// stage inputs (xin, min_) at time t -> buffer `cur`
mmvm_status run_prep_bufs(const DevTables& T, const StageBufs& B, int cur, const double* xin, const double* min_,
                          double t, mmvm_precision prec, hipStream_t st)
{
    void* tk = timing_begin(st);
    hipError_t e = launch_prep(T, B, cur, xin, min_, t, B.interact != 0, prec == MMVM_MIXED, st);
    timing_end(tk, "prep", st);
    return hip_status(e, "k_prep launch");
}

mmvm_status run_prep(const DevTables& T, Workspace& W, int cur, const double* xin, const double* min_, double t,
                     mmvm_precision prec, hipStream_t st)
{
    return run_prep_bufs(T, W.bufs, cur, xin, min_, t, prec, st);
}

}  // namespace mmvm

using namespace mmvm;

extern "C" {

const char* mmvm_status_string(mmvm_status s)
{
    switch (s) {
    case MMVM_OK: return "MMVM_OK";
    case MMVM_PENDING: return "MMVM_PENDING";
    case MMVM_EINVAL: return "MMVM_EINVAL";
    case MMVM_ENOMEM: return "MMVM_ENOMEM";
    case MMVM_EORDER: return "MMVM_EORDER";
    case MMVM_EZEROCIRC: return "MMVM_EZEROCIRC";
    case MMVM_EDEVICE: return "MMVM_EDEVICE";
    case MMVM_ENOTFOUND: return "MMVM_ENOTFOUND";
    case MMVM_EBUDGET: return "MMVM_EBUDGET";
    case MMVM_ENONFINITE: return "MMVM_ENONFINITE";
    }
    return "unknown";
}

mmvm_status mmvm_coeffs(int32_t order, int32_t kind, void* out, size_t out_bytes, size_t* needed_bytes)
{
    if (order < 0 || order > MMVM_MAX_ORDER) return MMVM_EORDER;
    const Tables& T = get_tables(order);
    size_t need = 0;
    if (kind == MMVM_TABLE_H) {
        int nmax = 3 * order + 1;
        size_t cnt = (size_t)(nmax + 1) * (nmax + 2) / 2;
        need = 2 * cnt * sizeof(double);
        if (needed_bytes) *needed_bytes = need;
        if (!out) return MMVM_OK;
        if (out_bytes < need) return MMVM_EINVAL;
        double* o = (double*)out;
        // H_1(a) = -Psi0(a + e2), H_2(a) = Psi0(a + e1), Psi0 nonzero only even-even
        for (int s = 0; s <= nmax; ++s)
            for (int a2 = 0; a2 <= s; ++a2) {
                int a1 = s - a2;
                size_t i = (size_t)tri(a1, a2);
                double h1 = 0.0, h2 = 0.0;
                if (a1 % 2 == 0 && a2 % 2 == 1) h1 = -T.t0_hi[tri(a1 / 2, (a2 + 1) / 2)];
                if (a1 % 2 == 1 && a2 % 2 == 0) h2 = T.t0_hi[tri((a1 + 1) / 2, a2 / 2)];
                o[i] = h1;
                o[cnt + i] = h2;
            }
        return MMVM_OK;
    }
    if (kind == MMVM_TABLE_FACTORS) {
        size_t cnt = (size_t)(order + 1) * (order + 1) * (order + 1);
        need = 2 * cnt * sizeof(double);
        if (needed_bytes) *needed_bytes = need;
        if (!out) return MMVM_OK;
        if (out_bytes < need) return MMVM_EINVAL;
        double* o = (double*)out;
        std::memcpy(o, T.f0_hi.data(), cnt * sizeof(double));
        std::memcpy(o + cnt, T.f1_hi.data(), cnt * sizeof(double));
        return MMVM_OK;
    }
    return MMVM_EINVAL;
}

mmvm_status mmvm_prepare(int32_t order)
{
    if (order < 0 || order > MMVM_MAX_ORDER) return MMVM_EORDER;
    const DevTables* T = nullptr;
    return device_tables(order, &T);
}

mmvm_status mmvm_rhs(const mmvm_problem* prob, double t, const double* x, const double* mom, double* dx,
                     double* dmom, mmvm_precision prec, void* stream)
{
    mmvm_status s = validate(prob);
    if (s != MMVM_OK) return s;
    if (!x || !mom || !dx || !dmom || !std::isfinite(t)) return MMVM_EINVAL;
    if (prec != MMVM_FP64 && prec != MMVM_MIXED) return MMVM_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    const DevTables* T = nullptr;
    if ((s = device_tables(prob->order, &T)) != MMVM_OK) return s;
    Workspace* W = workspace_for(st);
    if (!W) return MMVM_EDEVICE;
    std::lock_guard<std::mutex> lk(W->mu);
    if ((s = W->ensure(prob->n, prob->order, use_dd(prob->order, prec), prob->n == 1, st)) != MMVM_OK) return s;
    if ((s = W->set_params(prob->lambda0, nullptr, prob->nu, prob->n, st)) != MMVM_OK) return s;
    StageArgs A;
    std::memset(&A, 0, sizeof(A));
    A.mode = MODE_RHS;
    A.cur = 0;
    A.t_stage = t;
    A.t_next = t;
    A.dx = dx;
    A.dmom = dmom;
    if ((s = run_prep(*T, *W, 0, x, mom, t, prec, st)) != MMVM_OK) return s;
    return run_stage(*T, *W, prec, A, st);
}

mmvm_status mmvm_step(const mmvm_problem* prob, double t0, double dt, int64_t nsteps, double* x, double* mom,
                      mmvm_precision prec, void* stream)
{
    mmvm_status s = validate(prob);
    if (s != MMVM_OK) return s;
    if (!x || !mom || nsteps < 0 || !std::isfinite(t0) || !std::isfinite(dt)) return MMVM_EINVAL;
    if (prec != MMVM_FP64 && prec != MMVM_MIXED) return MMVM_EINVAL;
    if (nsteps == 0) return MMVM_OK;
    hipStream_t st = (hipStream_t)stream;
    const DevTables* T = nullptr;
    if ((s = device_tables(prob->order, &T)) != MMVM_OK) return s;
    Workspace* W = workspace_for(st);
    if (!W) return MMVM_EDEVICE;
    std::lock_guard<std::mutex> lk(W->mu);
    if ((s = W->ensure(prob->n, prob->order, use_dd(prob->order, prec), prob->n == 1, st)) != MMVM_OK) return s;
    if ((s = W->set_params(prob->lambda0, nullptr, prob->nu, prob->n, st)) != MMVM_OK) return s;
    return run_steps(*T, *W, t0, dt, nsteps, x, mom, prec, st);
}

mmvm_status mmvm_step_batch(const mmvm_batch* b, double t0, double dt, int64_t nsteps, double* x, double* mom,
                            mmvm_precision prec, void* stream)
{
    if (!b) return MMVM_EINVAL;
    if (b->n < 1 || b->order < 0 || b->order > MMVM_MAX_ORDER) return MMVM_EORDER;
    if (!b->nu || !b->lambda0) return MMVM_EINVAL;
    for (int j = 0; j < b->n; ++j) {
        if (!(b->nu[j] >= 0.0) || !std::isfinite(b->nu[j])) return MMVM_EINVAL;
        if (!(b->lambda0[j] > 0.0) || !std::isfinite(b->lambda0[j])) return MMVM_EINVAL;
    }
    if (!x || !mom || nsteps < 0 || !std::isfinite(t0) || !std::isfinite(dt)) return MMVM_EINVAL;
    if (prec != MMVM_FP64 && prec != MMVM_MIXED) return MMVM_EINVAL;
    if (nsteps == 0) return MMVM_OK;
    hipStream_t st = (hipStream_t)stream;
    const DevTables* T = nullptr;
    mmvm_status s;
    if ((s = device_tables(b->order, &T)) != MMVM_OK) return s;
    Workspace* W = workspace_for(st);
    if (!W) return MMVM_EDEVICE;
    std::lock_guard<std::mutex> lk(W->mu);
    if ((s = W->ensure(b->n, b->order, use_dd(b->order, prec), true, st)) != MMVM_OK) return s;
    if ((s = W->set_params(b->lambda0, b->nu, 0.0, b->n, st)) != MMVM_OK) return s;
    return run_steps(*T, *W, t0, dt, nsteps, x, mom, prec, st);
}

mmvm_status mmvm_sync(void* stream)
{
    hipStream_t st = (hipStream_t)stream;
    if (hipStreamSynchronize(st) != hipSuccess) return MMVM_EDEVICE;
    Workspace* W = workspace_for(st);
    if (!W) return MMVM_EDEVICE;
    std::lock_guard<std::mutex> lk(W->mu);
    int f = W->latched;
    W->latched = 0;
    if (W->flag_ptr) {
        int d = 0;
        if (hipMemcpy(&d, W->flag_ptr, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess) return MMVM_EDEVICE;
        f |= d;
        if (d && (hipMemsetAsync(W->flag_ptr, 0, sizeof(int), st) != hipSuccess || hipStreamSynchronize(st) != hipSuccess))
            return MMVM_EDEVICE;
    }
    if (f & 1) return MMVM_EZEROCIRC;
    if (f & 2) return MMVM_ENONFINITE;
    return MMVM_OK;
}

}  // extern "C"
