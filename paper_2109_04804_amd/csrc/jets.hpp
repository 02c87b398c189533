// Forward-mode jets used to evaluate the DGSEM fluxes together with their exact
// directional derivatives (R2 = R1'(w) sigma, Eq. DGSEM_wtt, and the Hessian
// term of the extended Jacobian, Eq. nonlinear_eqsys).
//
//   Dual<T>  a + b e                      one direction
//   Dual2<T> a + b e1 + c e2              two independent directions, no cross term
//   Jet5<T>  a + s e_s + d e_d + e e_e + sd e_s e_d   (e_s^2 = e_d^2 = e_e^2 = 0,
//            e_e e_s = e_e e_d = 0): directions sigma (s), dw (d), dsigma (e)
//            and the mixed second derivative along (sigma, dw).
//
// Non-smooth functions branch on the value part: |x| uses sign(a) with
// sign(0) = +1; max(x, y) returns x when a_x >= a_y.
#pragma once
#include <hip/hip_runtime.h>

#define HD __device__ __forceinline__

template <typename T> struct Dual { T a, b; };
template <typename T> struct Dual2 { T a, b, c; };
template <typename T> struct Jet5 { T a, s, d, e, sd; };

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

// ---------------------------------------------------------------- Jet5
template <typename T> HD Jet5<T> operator+(Jet5<T> x, Jet5<T> y) {
    return {x.a + y.a, x.s + y.s, x.d + y.d, x.e + y.e, x.sd + y.sd};
}
template <typename T> HD Jet5<T> operator-(Jet5<T> x, Jet5<T> y) {
    return {x.a - y.a, x.s - y.s, x.d - y.d, x.e - y.e, x.sd - y.sd};
}
template <typename T> HD Jet5<T> operator-(Jet5<T> x) { return {-x.a, -x.s, -x.d, -x.e, -x.sd}; }
template <typename T> HD Jet5<T> operator*(Jet5<T> x, Jet5<T> y) {
    return {x.a * y.a,
            x.a * y.s + x.s * y.a,
            x.a * y.d + x.d * y.a,
            x.a * y.e + x.e * y.a,
            x.a * y.sd + x.s * y.d + x.d * y.s + x.sd * y.a};
}
template <typename T> HD Jet5<T> operator*(Jet5<T> x, T k) { return {x.a * k, x.s * k, x.d * k, x.e * k, x.sd * k}; }
template <typename T> HD Jet5<T> operator*(T k, Jet5<T> x) { return x * k; }
template <typename T> HD Jet5<T> operator+(Jet5<T> x, T k) { return {x.a + k, x.s, x.d, x.e, x.sd}; }
// g(x) with g(a) = f0, g'(a) = f1, g''(a) = f2
template <typename T> HD Jet5<T> japply(Jet5<T> x, T f0, T f1, T f2) {
    return {f0, f1 * x.s, f1 * x.d, f1 * x.e, f1 * x.sd + f2 * x.s * x.d};
}
template <typename T> HD Jet5<T> jrecip(Jet5<T> x) {
    T r = T(1) / x.a;
    return japply(x, r, -r * r, T(2) * r * r * r);
}
template <typename T> HD Jet5<T> jsqrt(Jet5<T> x) {
    T s = sqrt(x.a);
    T d1 = T(0.5) / s;
    return japply(x, s, d1, -T(0.5) * d1 / x.a);
}
template <typename T> HD Jet5<T> jabs(Jet5<T> x) { return x.a >= T(0) ? x : -x; }
template <typename T> HD Jet5<T> jmax(Jet5<T> x, Jet5<T> y) { return x.a >= y.a ? x : y; }
template <typename T> HD T jval(Jet5<T> x) { return x.a; }

// constant of the jet type
template <typename S, typename T> HD S jconst(T k);
template <> HD double jconst<double, double>(double k) { return k; }
template <> HD float jconst<float, float>(float k) { return k; }
template <> HD Dual<double> jconst<Dual<double>, double>(double k) { return {k, 0.0}; }
template <> HD Dual<float> jconst<Dual<float>, float>(float k) { return {k, 0.0f}; }
template <> HD Dual2<double> jconst<Dual2<double>, double>(double k) { return {k, 0.0, 0.0}; }
template <> HD Dual2<float> jconst<Dual2<float>, float>(float k) { return {k, 0.0f, 0.0f}; }
template <> HD Jet5<double> jconst<Jet5<double>, double>(double k) { return {k, 0.0, 0.0, 0.0, 0.0}; }
template <> HD Jet5<float> jconst<Jet5<float>, float>(float k) { return {k, 0.0f, 0.0f, 0.0f, 0.0f}; }
