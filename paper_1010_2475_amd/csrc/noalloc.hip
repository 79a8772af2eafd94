// mmvm_rhs_noalloc: the right-hand side of mmvm_rhs with every workspace
// region taken from one file-scope device array instead of memory the
// library allocates.  For callers that cannot allocate (code under graph
// capture, tight serving loops, harnesses that forbid hipMalloc).
//
// The array's name is a host-side stand-in in host code; its device address
// is looked up once per device with hipGetSymbolAddress and only that address
// is passed to kernels.  Every call on a device shares that device's array:
// calls that overlap on one device (two streams, two threads) race.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <mutex>

#include "../../include/mmvm.h"
#include "api_internal.hpp"

namespace mmvm {
namespace {

constexpr size_t kScratchBytes = (size_t)MMVM_NOALLOC_SCRATCH_MB << 20;
constexpr int kMaxDevices = 64;
constexpr int kParamChunk = 128;  // core scales passed by value per launch

__device__ __align__(256) char scratch[kScratchBytes];

std::mutex g_mu;
char* g_scratch[kMaxDevices] = {};  // device address of `scratch` on each device, once looked up

// device address of this device's scratch array (looked up on first use)
mmvm_status scratch_ptr(char** out)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return MMVM_EDEVICE;
    if (dev < 0 || dev >= kMaxDevices) return MMVM_EDEVICE;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            report_hip_error(e, "hipGetSymbolAddress(scratch)");
            return MMVM_EDEVICE;
        }
        g_scratch[dev] = (char*)p;
    }
    *out = g_scratch[dev];
    return MMVM_OK;
}

// zeroes [p, p + n) (n a multiple of 8; a kernel rather than a memset, so the
// call can be captured)
__global__ __launch_bounds__(256) void k_zero(double* p, long n)
{
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) p[i] = 0.0;
}

struct ParamChunk {
    double lam0[kParamChunk];
};

// lambda_{j,0}^2 and nu for vortices j0 .. j0 + cnt - 1 (the host values travel
// as kernel arguments, so the caller's array is not read after the call)
__global__ __launch_bounds__(kParamChunk) void k_params(double* lam0sq, double* nuv, int j0, int cnt, double nu,
                                                      ParamChunk c)
{
    const int i = threadIdx.x;
    if (i < cnt) {
        lam0sq[j0 + i] = c.lam0[i] * c.lam0[i];
        nuv[j0 + i] = nu;
    }
}

}  // namespace
}  // namespace mmvm

using namespace mmvm;

extern "C" mmvm_status mmvm_rhs_noalloc(const mmvm_problem* prob, double t, const double* x, const double* mom,
                                        double* dx, double* dmom, mmvm_precision prec, void* stream)
{
    mmvm_status s = validate(prob);
    if (s != MMVM_OK) return s;
    if (!x || !mom || !dx || !dmom || !std::isfinite(t)) return MMVM_EINVAL;
    if (prec != MMVM_FP64 && prec != MMVM_MIXED) return MMVM_EINVAL;
    const DevTables* T = find_device_tables(prob->order);
    if (!T) return MMVM_ENOTFOUND;  // mmvm_prepare(order) has not run on this device
    const int N = prob->n;
    const bool solo = N == 1;
    const bool dd = use_dd(prob->order, prec);
    const size_t need = stage_layout(nullptr, N, prob->order, dd, solo, nullptr, nullptr, nullptr);
    if (need > kScratchBytes) return MMVM_EBUDGET;
    char* base = nullptr;
    if ((s = scratch_ptr(&base)) != MMVM_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    StageBufs B;
    double* par = nullptr;
    stage_layout(base, N, prob->order, dd, solo, &B, nullptr, &par);

    // the array keeps the previous call's contents: clear what this call uses
    const long nz = (long)(need / sizeof(double));
    int zb = (int)((nz + 255) / 256);
    if (zb > 2048) zb = 2048;
    hipLaunchKernelGGL(k_zero, dim3(zb), dim3(256), 0, st, (double*)base, nz);
    for (int j0 = 0; j0 < N; j0 += kParamChunk) {
        ParamChunk c;
        const int cnt = N - j0 < kParamChunk ? N - j0 : kParamChunk;
        std::memset(&c, 0, sizeof(c));
        for (int i = 0; i < cnt; ++i) c.lam0[i] = prob->lambda0[j0 + i];
        hipLaunchKernelGGL(k_params, dim3(1), dim3(kParamChunk), 0, st, par, par + N, j0, cnt, prob->nu, c);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        report_hip_error(e, "mmvm_rhs_noalloc set-up launch");
        return MMVM_EDEVICE;
    }

    StageArgs A;
    std::memset(&A, 0, sizeof(A));
    A.mode = MODE_RHS;
    A.cur = 0;
    A.t_stage = t;
    A.t_next = t;
    A.dx = dx;
    A.dmom = dmom;
    if ((s = run_prep_bufs(*T, B, 0, x, mom, t, prec, st)) != MMVM_OK) return s;
    const PairShape sh = pair_shape_known(prob->order, prec == MMVM_MIXED, N);
    return run_stage_bufs(*T, B, prec, A, st, &sh);
}
