// Double-double arithmetic (an unevaluated sum hi + lo of two doubles, ~106-bit
// significand), built from the error-free transformations TwoSum (Knuth) and
// TwoProd via fused multiply-add (Dekker's product with an FMA).  Every routine
// turns floating-point contraction off: a compiler-fused a*b + c inside them
// (HIP compiles with -ffp-contract=fast) would break the error-free
// transformations and leave only FP64 accuracy.  Used on the
// host for the coefficient tables and on the device for the self-interaction
// contraction at high order, where FP64 alone loses digits to cancellation.
#pragma once
#include <hip/hip_runtime.h>
#include <cmath>

namespace mmvm {

struct dd {
    double hi, lo;
};

__host__ __device__ inline dd dd_make(double h, double l = 0.0) { dd r; r.hi = h; r.lo = l; return r; }

__host__ __device__ inline dd two_sum(double a, double b)
{
#pragma clang fp contract(off)
    double s = a + b;
    double bb = s - a;
    double e = (a - (s - bb)) + (b - bb);
    return dd_make(s, e);
}

__host__ __device__ inline dd quick_two_sum(double a, double b)
{
#pragma clang fp contract(off)
    double s = a + b;
    double e = b - (s - a);
    return dd_make(s, e);
}

__host__ __device__ inline dd two_prod(double a, double b)
{
#pragma clang fp contract(off)
    double p = a * b;
    double e = fma(a, b, -p);
    return dd_make(p, e);
}

__host__ __device__ inline dd dd_add(dd a, dd b)
{
#pragma clang fp contract(off)
    dd s = two_sum(a.hi, b.hi);
    dd t = two_sum(a.lo, b.lo);
    s.lo += t.hi;
    s = quick_two_sum(s.hi, s.lo);
    s.lo += t.lo;
    return quick_two_sum(s.hi, s.lo);
}

__host__ __device__ inline dd dd_neg(dd a) { return dd_make(-a.hi, -a.lo); }
__host__ __device__ inline dd dd_sub(dd a, dd b) { return dd_add(a, dd_neg(b)); }

__host__ __device__ inline dd dd_mul(dd a, dd b)
{
#pragma clang fp contract(off)
    dd p = two_prod(a.hi, b.hi);
    p.lo += a.hi * b.lo + a.lo * b.hi;
    return quick_two_sum(p.hi, p.lo);
}

__host__ __device__ inline dd dd_mul_d(dd a, double b)
{
#pragma clang fp contract(off)
    dd p = two_prod(a.hi, b);
    p.lo += a.lo * b;
    return quick_two_sum(p.hi, p.lo);
}

// acc += a * b
__host__ __device__ inline dd dd_fma(dd acc, dd a, dd b) { return dd_add(acc, dd_mul(a, b)); }

__host__ __device__ inline dd dd_div(dd a, dd b)
{
#pragma clang fp contract(off)
    double q1 = a.hi / b.hi;
    dd r = dd_sub(a, dd_mul_d(b, q1));
    double q2 = r.hi / b.hi;
    r = dd_sub(r, dd_mul_d(b, q2));
    double q3 = r.hi / b.hi;
    dd q = quick_two_sum(q1, q2);
    return dd_add(q, dd_make(q3));
}

}  // namespace mmvm
