// Small device helpers shared by the kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>
#include <utility>

namespace mmvm {

__host__ __device__ __forceinline__ constexpr int ctri(int a, int b) { return (a + b) * (a + b + 1) / 2 + b; }

template <int B, int E, typename F>
__device__ __forceinline__ void sfor(F&& f)
{
    if constexpr (B < E) {
        f(std::integral_constant<int, B>());
        sfor<B + 1, E>(f);
    }
}

__device__ __forceinline__ int shell_of(int k)
{
    int s = (int)((sqrt(8.0 * k + 1.0) - 1.0) * 0.5);
    while ((s + 1) * (s + 2) / 2 <= k) ++s;
    while (s * (s + 1) / 2 > k) --s;
    return s;
}

}  // namespace mmvm
