// device_math.h -- arithmetic helpers shared by the solver and the stats kernels.
#pragma once

#include <hip/hip_runtime.h>

namespace gamer {

template <typename T>
struct Consts {
    T g, gm1, igm1, theta, half;
    T gq;  // gamma (gamma - 1) / 2: (rho c)^2 = gq (2 rho E - |m|^2)
};

// Reciprocal and square root.  float: the hardware instructions (about 1 ulp,
// well inside the FP32 path's tolerance).  double: the hardware estimate
// refined by Newton steps to within a few ulp of the IEEE result, without the
// range scaling of the IEEE expansions (operands here are normal numbers).
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float sqrt_(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double rcp(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}
__device__ __forceinline__ float rsq(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double rsq(double x) {
    // two Newton steps y <- y + y (1/2 - x y^2 / 2) on the hardware estimate
    double y = __builtin_amdgcn_rsq(x);
    const double hx = 0.5 * x;
    double e = fma(-hx * y, y, 0.5);
    y = fma(y, e, y);
    e = fma(-hx * y, y, 0.5);
    return fma(y, e, y);
}
__device__ __forceinline__ double sqrt_(double x) {
    // Goldschmidt iteration on the reciprocal square root estimate
    const double y = __builtin_amdgcn_rsq(x);
    double g = x * y, h = 0.5 * y;
    double r = fma(-g, h, 0.5);
    g = fma(g, r, g);
    h = fma(h, r, h);
    r = fma(-g, h, 0.5);
    g = fma(g, r, g);
    h = fma(h, r, h);
    const double d = fma(-g, g, x);
    g = fma(d, h, g);
    return x > 0.0 ? g : (x == 0.0 ? 0.0 : __builtin_nan(""));
}

// |u| + |v| + |w| + 3 c_s of a conserved state in the working precision, or NaN
// when the state is not physical (rho <= 0 or p <= 0) or not finite: such a
// state has no sound speed, and the NaN carries through the maxima below to
// the time step instead of being dropped.  The solver epilogue and the
// stand-alone stats kernel both use this function, so their per-group maxima
// agree bitwise.
template <typename T>
__device__ __forceinline__ T signal_speed(T r, T mx, T my, T mz, T e, const Consts<T> &c) {
    const T ir = rcp(r);
    const T u = mx * ir, v = my * ir, w = mz * ir;
    const T p = c.gm1 * (e - c.half * (mx * u + my * v + mz * w));
    const T cs = sqrt_(c.g * p * ir);
    const T s = fabs(u) + fabs(v) + fabs(w) + T(3) * cs;
    return (r > T(0) && p > T(0) && isfinite(s)) ? s : T(__builtin_nan(""));
}

// Maximum that keeps a NaN of either operand (fmax drops it).
__device__ __forceinline__ double max_nan(double a, double b) { return (a > b || a != a) ? a : b; }

template <typename T>
__device__ __forceinline__ Consts<T> make_consts(double gamma, double theta) {
    return Consts<T>{T(gamma), T(gamma - 1.0), T(1.0 / (gamma - 1.0)), T(theta), T(0.5),
                     T(0.5 * gamma * (gamma - 1.0))};
}

}  // namespace gamer
