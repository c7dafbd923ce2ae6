// scaled.hpp -- complex numbers with a separate binary exponent, for the
// products over many slabs of the multilevel estimators (arXiv 1309.3859,
// Sec. II.C.2-3), whose averages have modulus below one.
#pragma once

#include <hip/hip_runtime.h>

namespace u1ml {

// value = (re + i im) 2^ex, max(|re|, |im|) >= 2^-600 or 0
struct sc {
    double re, im;
    int ex;
};

__device__ inline sc sc_norm(double re, double im, int ex)
{
    const double m = fmax(fabs(re), fabs(im));
    if (m == 0.0 || !isfinite(m)) return sc{re, im, 0};
    const int k = ilogb(m);
    return sc{ldexp(re, -k), ldexp(im, -k), ex + k};
}

// The mantissa is renormalised only once its magnitude falls below 2^-600:
// scaling by a power of two commutes with rounding while values stay normal,
// so the result equals renormalising after every product, bit for bit.
__device__ inline sc sc_lazy(double re, double im, int ex)
{
    if (fmax(fabs(re), fabs(im)) < 0x1p-600) return sc_norm(re, im, ex);
    return sc{re, im, ex};
}

__device__ inline sc sc_mul(sc a, double2 b) { return sc_lazy(a.re * b.x - a.im * b.y, a.re * b.y + a.im * b.x, a.ex); }

__device__ inline sc sc_mul(sc a, sc b)
{
    return sc_lazy(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re, a.ex + b.ex);
}

// binary exponent of the value (that of max(|re|, |im|), plus ex); kNoExp for
// zero or a non-finite value
constexpr int kNoExp = -2147483647 - 1;
__device__ inline int sc_exp(sc a)
{
    const double m = fmax(fabs(a.re), fabs(a.im));
    if (m == 0.0 || !isfinite(m)) return kNoExp;
    return a.ex + ilogb(m);
}

// the value times 2^-E as a plain complex double (exact unless it leaves the
// normal range)
__device__ inline double2 sc_rel(sc a, int E)
{
    long long k = (long long)a.ex - E;
    k = k < -2200 ? -2200 : (k > 2200 ? 2200 : k);
    return make_double2(ldexp(a.re, (int)k), ldexp(a.im, (int)k));
}

}  // namespace u1ml
