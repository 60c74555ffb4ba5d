// primitives.h -- device-side pieces shared by the generation and
// application kernels: address-space casts, the rotation generator and the
// rotation (Section 3.4, eqs. (giv), (giv1)).
//
// Rounding: every operation is rounded on its own (-ffp-contract=off);
// fma only where written; sqrt and division are IEEE.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bdu {

#define GLOBAL __attribute__((address_space(1)))
#define CONSTANT __attribute__((address_space(4)))
#define LOCAL __attribute__((address_space(3)))

// Pointers read from a descriptor are generic; the kernels know which memory
// they point to.  Global pointers give global (not flat) memory instructions,
// constant pointers with a uniform index give scalar loads.
template <typename T>
__device__ __forceinline__ GLOBAL T *gptr(T *p)
{
    return (GLOBAL T *)(uintptr_t)p;
}
template <typename T>
__device__ __forceinline__ const CONSTANT T *kptr(const T *p)
{
    return (const CONSTANT T *)(uintptr_t)p;
}

// ---- primitives (eq. giv1) -------------------------------------------------

// Rotation generator: mode 1 gives [c -s; s c][a;b] = [0;r], mode 2 gives
// [r;0]; r = +sqrt(a^2 + b^2) with an exact power-of-two scaling when the
// larger magnitude is extreme; identity when the target is already zero.
//
// Written with selects only: both the identity and the general result are
// computed (the general one may be NaN when a = b = 0 and is then discarded),
// so a wavefront runs one straight sequence whatever its lanes' data.
template <int MODE>
__device__ __forceinline__ void givens_m(double a, double b, double &c, double &s, double &r)
{
    constexpr bool m1 = MODE == 1;
    const double fa = fabs(a), fb = fabs(b);
    const double big = fa > fb ? fa : fb;
    const bool hi = big > 0x1p500, lo = big < 0x1p-500;
    const double sc = hi ? 0x1p-600 : (lo ? 0x1p600 : 1.0);
    const double unsc = hi ? 0x1p600 : (lo ? 0x1p-600 : 1.0);
    const double as = a * sc, bs = b * sc;
    const double rs = sqrt(fma(as, as, bs * bs));
    const double p = (m1 ? bs : as) / rs, q = (m1 ? as : bs) / rs;
    const bool ident = (m1 ? a : b) == 0.0;
    c = ident ? 1.0 : p;
    s = ident ? 0.0 : (m1 ? q : -q);
    r = ident ? (m1 ? b : a) : rs * unsc;
}

__device__ __forceinline__ void givens(double a, double b, int mode, double &c, double &s, double &r)
{
    if (mode == 1)
        givens_m<1>(a, b, c, s, r);
    else
        givens_m<2>(a, b, c, s, r);
}

__device__ __forceinline__ void rot(double c, double s, double &x, double &y)
{
    double x0 = x, y0 = y;
    x = fma(c, x0, -(s * y0));
    y = fma(s, x0, c * y0);
}

}  // namespace bdu
