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

// The same generator, faster when the magnitudes of a and b lie in
// [2^-370, 2^370] on every active lane of the wavefront (a wave-uniform
// test; otherwise the general form above runs).  In that range no scaling
// applies, the target is nonzero, r^2 = a^2 + b^2 is at least 2^-740, and
// both quotients and 1/r are normal numbers, so the IEEE square root and the
// two IEEE divisions by r reduce to their core sequences with the same
// correctly rounded results: the square root as an rsq estimate with two
// Newton-Raphson corrections, each division as the reciprocal refined twice,
// the product and one residual correction.  Their scaling and special-value
// steps only change operands outside the range.  The two divisions share
// the reciprocal of r.
template <int MODE>
__device__ __forceinline__ void givens_fast(double a, double b, double &c, double &s, double &r)
{
    const double fa = fabs(a), fb = fabs(b);
    const bool in = fa >= 0x1p-370 && fa <= 0x1p370 && fb >= 0x1p-370 && fb <= 0x1p370;
    if (!__all(in)) {
        givens_m<MODE>(a, b, c, s, r);
        return;
    }
    constexpr bool m1 = MODE == 1;
    const double x = fma(a, a, b * b);
    // square root of x
    const double y = __builtin_amdgcn_rsq(x);
    double g = x * y, h = y * 0.5;
    const double t = fma(-h, g, 0.5);
    g = fma(g, t, g);
    h = fma(h, t, h);
    double d = fma(-g, g, x);
    g = fma(d, h, g);
    d = fma(-g, g, x);
    g = fma(d, h, g);
    const double rs = g;
    // 1/rs, refined twice
    double rc = __builtin_amdgcn_rcp(rs);
    double e = fma(-rs, rc, 1.0);
    rc = fma(rc, e, rc);
    e = fma(-rs, rc, 1.0);
    rc = fma(rc, e, rc);
    auto quot = [&](double n) {
        const double q0 = n * rc;
        const double rem = fma(-rs, q0, n);
        return fma(rem, rc, q0);
    };
    const double p = quot(m1 ? b : a), q = quot(m1 ? a : b);
    c = p;
    s = m1 ? q : -q;
    r = rs;
}

__device__ __forceinline__ void givens(double a, double b, int mode, double &c, double &s, double &r)
{
    if (mode == 1)
        givens_fast<1>(a, b, c, s, r);
    else
        givens_fast<2>(a, b, c, s, r);
}

__device__ __forceinline__ void rot(double c, double s, double &x, double &y)
{
    double x0 = x, y0 = y;
    x = fma(c, x0, -(s * y0));
    y = fma(s, x0, c * y0);
}

}  // namespace bdu
