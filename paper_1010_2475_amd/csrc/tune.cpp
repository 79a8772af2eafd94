// Launch-shape autotuner.  The first launch of a tunable kernel for a new key
// (order, precision, vortex count rounded up to a power of two) times every
// candidate shape on the caller's stream, on the caller's own inputs, and the
// fastest one is kept for the rest of the process: later launches with that
// key pay nothing, and a key always gets the same shape within a process (so
// the same bits).  With tuning off the fixed default shape runs.
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "api_internal.hpp"

namespace mmvm {

namespace {

struct PairEntry {
    PairShape shape;
    double us = 0.0;      // average launch time of the chosen shape
    double us_def = 0.0;  // ... and of the default shape
    int candidates = 0;
};

std::mutex g_mu;
std::map<std::tuple<int, int, int>, PairEntry> g_pair;  // (order, f32, N bucket)
int g_enabled = -1;                                    // -1: not yet read from MMVM_AUTOTUNE

bool enabled_locked()
{
    if (g_enabled < 0) {
        const char* e = std::getenv("MMVM_AUTOTUNE");
        g_enabled = (e && e[0] == '0') ? 0 : 1;
    }
    return g_enabled == 1;
}

int bucket(int n)
{
    int b = 1;
    while (b < n) b <<= 1;
    return b;
}

// average time of `reps` launches of one shape, after one untimed launch;
// negative on a launch error
double time_pair(const DevTables& T, const StageBufs& B, int cur, bool f32, PairShape sh, hipStream_t st,
                 hipEvent_t e0, hipEvent_t e1)
{
    const int reps = 3;
    if (launch_pair_shape(T, B, cur, f32, sh, st) != hipSuccess) return -1.0;
    if (hipEventRecord(e0, st) != hipSuccess) return -1.0;
    for (int r = 0; r < reps; ++r)
        if (launch_pair_shape(T, B, cur, f32, sh, st) != hipSuccess) return -1.0;
    if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) return -1.0;
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return -1.0;
    return 1e3 * (double)ms / reps;
}

}  // namespace

PairShape pair_shape_known(int M, bool f32, int N)
{
    std::lock_guard<std::mutex> lk(g_mu);
    if (!enabled_locked()) return PairShape();
    auto it = g_pair.find(std::make_tuple(M, f32 ? 1 : 0, bucket(N)));
    return it == g_pair.end() ? PairShape() : it->second.shape;
}

PairShape pair_shape_for(const DevTables& T, const StageBufs& B, int cur, bool f32, hipStream_t st)
{
    const PairShape def;
    if (T.M > kMaxPairOrder) return def;  // the runtime-order kernel has one shape
    std::lock_guard<std::mutex> lk(g_mu);
    if (!enabled_locked()) return def;
    const auto key = std::make_tuple(T.M, f32 ? 1 : 0, bucket(B.N));
    auto it = g_pair.find(key);
    if (it != g_pair.end()) return it->second.shape;

    // the candidates: up to four wavefronts per workgroup, a target's sources
    // split over 1, 2 or 4 of them (each keeping at least 32 sources)
    // (for the mixed precision also the FP64 variant of the unrolled kernel: a
    // key may run FP64 wherever that is faster)
    // and each of those with the far-field chunks split off to the multipole kernel
    // The far split decides per 64-source chunk at run time, so it costs a dense
    // field only its mask (one ballot and byte per chunk) and a scan of that mask,
    // while a key (tuned on one geometry) may later see a dilute one: from
    // kPairFarAlwaysN vortices every candidate splits the far field off.
    // MMVM_PAIR_FAR=0 / 1 restricts the candidates to either form.
    int far_lo = 0, far_hi = B.far_mask ? 1 : 0;
    if (far_hi && B.N >= kPairFarAlwaysN) far_lo = 1;
    if (const char* f = std::getenv("MMVM_PAIR_FAR")) {
        if (f[0] == '0') far_lo = far_hi = 0;
        else if (f[0] == '1' && B.far_mask) far_lo = far_hi = 1;
    }
    std::vector<PairShape> cand;
    for (int far = far_lo; far <= far_hi; ++far)
        for (int f64 = (f32 && T.M > kPairF32MaxOrder) ? 1 : 0; f64 <= (f32 ? 1 : 0); ++f64)
            for (int split = 1; split <= 4; split <<= 1)
                for (int tpb = 1; tpb <= 4; tpb <<= 1) {
                    PairShape s;
                    s.split = split;
                    s.tpb = tpb;
                    s.f64 = f64;
                    s.far = far;
                    if (pair_shape_valid(s) && (split == 1 || B.N >= 32 * split)) cand.push_back(s);
                }
    // the few-vortex kernel (16 lanes per pair, FP64)
    if (B.N >= 2 && !B.rank) {
        PairShape s;
        s.kind = 1;
        s.groups = pair_split_groups(B.N);
        if (s.groups == 1 || B.p_part) cand.push_back(s);
    }
    // the tuning launches are not the caller's timed kernel
    TimingSlot* saved = timing_slot();
    timing_slot() = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    PairEntry best;
    best.shape = def;
    best.us = -1.0;
    if (hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess) {
        for (const PairShape& s : cand) {
            const double us = time_pair(T, B, cur, f32, s, st, e0, e1);
            if (us < 0.0) continue;
            ++best.candidates;
            if (s.kind == def.kind && s.split == def.split && s.tpb == def.tpb && s.f64 == def.f64 && s.far == def.far)
                best.us_def = us;
            if (best.us < 0.0 || us < best.us) {
                best.us = us;
                best.shape = s;
            }
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    timing_slot() = saved;
    (void)hipGetLastError();
    if (best.candidates == 0) return def;  // nothing could be timed: leave the key untuned
    g_pair[key] = best;
    return best.shape;
}

}  // namespace mmvm

using namespace mmvm;

extern "C" {

mmvm_status mmvm_autotune_enable(int32_t on)
{
    std::lock_guard<std::mutex> lk(g_mu);
    g_enabled = on ? 1 : 0;
    return MMVM_OK;
}

mmvm_status mmvm_autotune_report(char* buf, size_t cap, size_t* needed)
{
    std::string out;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        char line[256];
        for (const auto& kv : g_pair) {
            const PairEntry& e = kv.second;
            std::snprintf(line, sizeof(line),
                          "pair order=%d prec=%s n<=%d kind=%d split=%d tpb=%d groups=%d f64=%d far=%d us=%.3f "
                          "default_us=%.3f candidates=%d\n",
                          std::get<0>(kv.first), std::get<1>(kv.first) ? "mixed" : "fp64", std::get<2>(kv.first),
                          e.shape.kind, e.shape.split, e.shape.tpb, e.shape.groups, e.shape.f64, e.shape.far, e.us,
                          e.us_def, e.candidates);
            out += line;
        }
    }
    if (needed) *needed = out.size() + 1;
    if (!buf) return MMVM_OK;
    if (cap < out.size() + 1) return MMVM_EINVAL;
    std::memcpy(buf, out.c_str(), out.size() + 1);
    return MMVM_OK;
}

}  // extern "C"
