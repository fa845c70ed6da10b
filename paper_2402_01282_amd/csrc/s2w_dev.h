// Device helpers shared by the FP64 and mixed-precision kernels.
#pragma once

#include <hip/hip_runtime.h>

namespace s2w {

__device__ __forceinline__ void powexp(double x, int p, double &mt, int &et)
{
    mt = 1.0;
    et = 0;
    if (p == 0) return;
    int bx;
    double bm = frexp(x, &bx);
    while (p) {
        if (p & 1) {
            int t;
            mt = frexp(mt * bm, &t);
            et += t + bx;
        }
        int t2;
        bm = frexp(bm * bm, &t2);
        bx = 2 * bx + t2;
        p >>= 1;
    }
}

// d^{l0}_mn(theta) as e * 2^(512 k), |e| in [2^-256, 2^256) or 0.
__device__ __forceinline__ void start_value(double mant, int ex, int p1, int p2, double ch, double sh,
                                   double ceps, double seps, double &e, int &k)
{
    if ((ch == 0.0 && p1 > 0) || (sh == 0.0 && p2 > 0) || mant == 0.0) {
        e = 0.0;
        k = 0;
        return;
    }
    double mc, ms;
    int ec, es;
    powexp(ch, p1, mc, ec);
    powexp(sh, p2, ms, es);
    mc *= fma((double)p1, ceps, 1.0);
    ms *= fma((double)p2, seps, 1.0);
    const double v = mant * mc * ms;
    const int E = ex + ec + es;
    int kk = (E + 256) >> 9;
    if (kk > 0) kk = 0;
    e = ldexp(v, E - 512 * kk);
    k = kk;
}

template <typename T>
struct V2;
template <>
struct V2<double> {
    typedef double2 t;
};
template <>
struct V2<float> {
    typedef float2 t;
};
template <typename T>
__device__ __forceinline__ typename V2<T>::t mk2(T x, T y)
{
    typename V2<T>::t v;
    v.x = x;
    v.y = y;
    return v;
}

}  // namespace s2w
