// Forward-mode jets used to evaluate the DGSEM fluxes together with their exact
// directional derivatives (R2 = R1'(w) sigma, Eq. DGSEM_wtt, and the Hessian
// term of the extended Jacobian, Eq. nonlinear_eqsys).
//
//   Dual<T>  a + b e                      one direction
//   Dual2<T> a + b e1 + c e2              two independent directions, no cross term
//   HDual<T> a + s e_s + d e_d + m e_s e_d (hyper-dual, e_s^2 = e_d^2 = 0): for
//            x = w + sigma e_s + dw e_d + dsigma e_s e_d the e_d part of F(x) is
//            F'(w) dw and the e_s e_d part F'(w) dsigma + F''(w)[sigma, dw]: both
//            JVP terms (with the Hessian term) in four components.
//
// Non-smooth functions branch on the value part: |x| uses sign(a) with
// sign(0) = +1; max(x, y) returns x when a_x >= a_y.
#pragma once
#include <hip/hip_runtime.h>

#define HD __device__ __forceinline__

template <typename T> struct Dual { T a, b; };
template <typename T> struct Dual2 { T a, b, c; };
template <typename T> struct HDual { T a, s, d, m; };

// ---------------------------------------------------------------- plain scalars
template <typename T> HD T jrecip(T x) { return T(1) / x; }
template <typename T> HD T jsqrt(T x) { return sqrt(x); }
template <typename T> HD T jabs(T x) { return x >= T(0) ? x : -x; }
template <typename T> HD T jmax(T x, T y) { return x >= y ? x : y; }
template <typename T> HD T jval(T x) { return x; }

// ---------------------------------------------------------------- Dual
template <typename T> HD Dual<T> operator+(Dual<T> x, Dual<T> y) { return {x.a + y.a, x.b + y.b}; }
template <typename T> HD Dual<T> operator-(Dual<T> x, Dual<T> y) { return {x.a - y.a, x.b - y.b}; }
template <typename T> HD Dual<T> operator-(Dual<T> x) { return {-x.a, -x.b}; }
template <typename T> HD Dual<T> operator*(Dual<T> x, Dual<T> y) { return {x.a * y.a, x.a * y.b + x.b * y.a}; }
template <typename T> HD Dual<T> operator*(Dual<T> x, T k) { return {x.a * k, x.b * k}; }
template <typename T> HD Dual<T> operator*(T k, Dual<T> x) { return {x.a * k, x.b * k}; }
template <typename T> HD Dual<T> operator+(Dual<T> x, T k) { return {x.a + k, x.b}; }
template <typename T> HD Dual<T> jrecip(Dual<T> x) { T r = T(1) / x.a; return {r, -r * r * x.b}; }
template <typename T> HD Dual<T> jsqrt(Dual<T> x) { T s = sqrt(x.a); return {s, x.b * (T(0.5) / s)}; }
template <typename T> HD Dual<T> jabs(Dual<T> x) { return x.a >= T(0) ? x : -x; }
template <typename T> HD Dual<T> jmax(Dual<T> x, Dual<T> y) { return x.a >= y.a ? x : y; }
template <typename T> HD T jval(Dual<T> x) { return x.a; }

// ---------------------------------------------------------------- Dual2
template <typename T> HD Dual2<T> operator+(Dual2<T> x, Dual2<T> y) { return {x.a + y.a, x.b + y.b, x.c + y.c}; }
template <typename T> HD Dual2<T> operator-(Dual2<T> x, Dual2<T> y) { return {x.a - y.a, x.b - y.b, x.c - y.c}; }
template <typename T> HD Dual2<T> operator-(Dual2<T> x) { return {-x.a, -x.b, -x.c}; }
template <typename T> HD Dual2<T> operator*(Dual2<T> x, Dual2<T> y) {
    return {x.a * y.a, x.a * y.b + x.b * y.a, x.a * y.c + x.c * y.a};
}
template <typename T> HD Dual2<T> operator*(Dual2<T> x, T k) { return {x.a * k, x.b * k, x.c * k}; }
template <typename T> HD Dual2<T> operator*(T k, Dual2<T> x) { return {x.a * k, x.b * k, x.c * k}; }
template <typename T> HD Dual2<T> operator+(Dual2<T> x, T k) { return {x.a + k, x.b, x.c}; }
template <typename T> HD Dual2<T> jrecip(Dual2<T> x) {
    T r = T(1) / x.a; T d = -r * r;
    return {r, d * x.b, d * x.c};
}
template <typename T> HD Dual2<T> jsqrt(Dual2<T> x) {
    T s = sqrt(x.a); T d = T(0.5) / s;
    return {s, d * x.b, d * x.c};
}
template <typename T> HD Dual2<T> jabs(Dual2<T> x) { return x.a >= T(0) ? x : -x; }
template <typename T> HD Dual2<T> jmax(Dual2<T> x, Dual2<T> y) { return x.a >= y.a ? x : y; }
template <typename T> HD T jval(Dual2<T> x) { return x.a; }

// ---------------------------------------------------------------- HDual
template <typename T> HD HDual<T> operator+(HDual<T> x, HDual<T> y) { return {x.a + y.a, x.s + y.s, x.d + y.d, x.m + y.m}; }
template <typename T> HD HDual<T> operator-(HDual<T> x, HDual<T> y) { return {x.a - y.a, x.s - y.s, x.d - y.d, x.m - y.m}; }
template <typename T> HD HDual<T> operator-(HDual<T> x) { return {-x.a, -x.s, -x.d, -x.m}; }
template <typename T> HD HDual<T> operator*(HDual<T> x, HDual<T> y) {
    return {x.a * y.a, x.a * y.s + x.s * y.a, x.a * y.d + x.d * y.a, x.a * y.m + x.s * y.d + x.d * y.s + x.m * y.a};
}
template <typename T> HD HDual<T> operator*(HDual<T> x, T k) { return {x.a * k, x.s * k, x.d * k, x.m * k}; }
template <typename T> HD HDual<T> operator*(T k, HDual<T> x) { return x * k; }
template <typename T> HD HDual<T> operator+(HDual<T> x, T k) { return {x.a + k, x.s, x.d, x.m}; }
// g(x) with g(a) = f0, g'(a) = f1, g''(a) = f2
template <typename T> HD HDual<T> japply(HDual<T> x, T f0, T f1, T f2) {
    return {f0, f1 * x.s, f1 * x.d, f1 * x.m + f2 * x.s * x.d};
}
template <typename T> HD HDual<T> jrecip(HDual<T> x) {
    T r = T(1) / x.a;
    return japply(x, r, -r * r, T(2) * r * r * r);
}
template <typename T> HD HDual<T> jsqrt(HDual<T> x) {
    T s = sqrt(x.a);
    T d1 = T(0.5) / s;
    return japply(x, s, d1, -T(0.5) * d1 / x.a);
}
template <typename T> HD HDual<T> jabs(HDual<T> x) { return x.a >= T(0) ? x : -x; }
template <typename T> HD HDual<T> jmax(HDual<T> x, HDual<T> y) { return x.a >= y.a ? x : y; }
template <typename T> HD T jval(HDual<T> x) { return x.a; }

// components of a jet in member order (the inverse of building it from x[0..])
template <typename T> HD void jet_split(T v, T* x) { x[0] = v; }
template <typename T> HD void jet_split(Dual<T> v, T* x) { x[0] = v.a; x[1] = v.b; }
template <typename T> HD void jet_split(Dual2<T> v, T* x) { x[0] = v.a; x[1] = v.b; x[2] = v.c; }
template <typename T> HD void jet_split(HDual<T> v, T* x) { x[0] = v.a; x[1] = v.s; x[2] = v.d; x[3] = v.m; }

// constant of the jet type
template <typename S, typename T> HD S jconst(T k);
template <> HD double jconst<double, double>(double k) { return k; }
template <> HD float jconst<float, float>(float k) { return k; }
template <> HD Dual<double> jconst<Dual<double>, double>(double k) { return {k, 0.0}; }
template <> HD Dual<float> jconst<Dual<float>, float>(float k) { return {k, 0.0f}; }
template <> HD Dual2<double> jconst<Dual2<double>, double>(double k) { return {k, 0.0, 0.0}; }
template <> HD Dual2<float> jconst<Dual2<float>, float>(float k) { return {k, 0.0f, 0.0f}; }
template <> HD HDual<double> jconst<HDual<double>, double>(double k) { return {k, 0.0, 0.0, 0.0}; }
template <> HD HDual<float> jconst<HDual<float>, float>(float k) { return {k, 0.0f, 0.0f, 0.0f}; }
