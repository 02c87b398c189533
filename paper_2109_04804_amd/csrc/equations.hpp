// Physical and numerical fluxes on device, templated on the scalar/jet type S.
//
// Numerical flux (Eq. Riemann, textbook 1/2 on the dissipation):
//   f*(wL, wR; +e_m) = (F_m(wL) + F_m(wR))/2 + lambda (wL - wR)/2
// lambda: central 0, upwind |a_m|, lf a global constant, rusanov
// max(|v_m,L| + c_L/eps, |v_m,R| + c_R/eps) with c = sqrt(gamma p / rho).
// lf_literal (Euler): Eq. Riemann as printed, f* = (F_m(wL) + F_m(wR))/2 + lambda_v (wL - wR)
// with no 1/2 and the diagonal lambda of the Euler set-up (Sec. 4.1.2), 1/eps on density and
// energy, 1 on the momenta.
// Euler is the eps-scaled system of Eq. Euler: momentum flux carries p/eps^2,
// p = (gamma - 1)(E - eps^2/2 |rho v|^2 / rho).
#pragma once
#include "jets.hpp"

enum { FLUX_CENTRAL = 0, FLUX_UPWIND = 1, FLUX_LF = 2, FLUX_RUSANOV = 3, FLUX_LF_LITERAL = 4 };

template <typename T> struct EqParams {
    T adv[3];
    T lam;      // constant lambda (lf)
    T nu;       // viscosity (Burgers)
    T gm1;      // gamma - 1
    T gamma;
    T half_eps2;
    T inv_eps;
    T inv_eps2;
    T mu;        // Navier-Stokes: dynamic viscosity
    T kappa;     // heat conductivity c_p mu / Pr
    T gam_eps2;  // 1 / R = gamma eps^2 (T = p / (rho R))
    T eta;       // BR2 stabilisation
    int flux;
};

template <int D> struct AdvectionEq {
    static constexpr int NV = 1;
    static constexpr bool VISC = false;
    static constexpr bool NS = false;
    template <class S, class T> HD static void flux_dir(const S* w, int m, S* F, const EqParams<T>& p) {
        F[0] = w[0] * p.adv[m];
    }
    template <class S, class T> HD static void flux_all(const S* w, S (*F)[NV], const EqParams<T>& p) {
#pragma unroll
        for (int m = 0; m < D; ++m) F[m][0] = w[0] * p.adv[m];
    }
    template <class S, class T> HD static S wave_speed(const S* w, int m, const EqParams<T>& p) {
        return jconst<S, T>(jabs(p.adv[m]));
    }
};

template <int D> struct BurgersEq {   // inviscid part u^2/2 per direction; the operator adds -nu q (BR1)
    static constexpr int NV = 1;
    static constexpr bool VISC = true;
    static constexpr bool NS = false;
    template <class S, class T> HD static void flux_dir(const S* w, int m, S* F, const EqParams<T>& p) {
        F[0] = w[0] * w[0] * T(0.5);
    }
    template <class S, class T> HD static void flux_all(const S* w, S (*F)[NV], const EqParams<T>& p) {
        S f = w[0] * w[0] * T(0.5);
#pragma unroll
        for (int m = 0; m < D; ++m) F[m][0] = f;
    }
    template <class S, class T> HD static S wave_speed(const S* w, int m, const EqParams<T>& p) {
        return jabs(w[0]);
    }
};

template <int D> struct EulerEq {
    static constexpr int NV = D + 2;
    static constexpr bool VISC = false;
    static constexpr bool NS = false;
    template <class S, class T> HD static S pressure(const S* w, S irho, const EqParams<T>& p) {
        S m2 = w[1] * w[1];
#pragma unroll
        for (int k = 1; k < D; ++k) m2 = m2 + w[1 + k] * w[1 + k];
        return (w[D + 1] - m2 * irho * p.half_eps2) * p.gm1;
    }
    template <class S, class T> HD static void flux_dir(const S* w, int m, S* F, const EqParams<T>& p) {
        S irho = jrecip(w[0]);
        S pr = pressure(w, irho, p);
        S vm = w[1 + m] * irho;
        F[0] = w[1 + m];
#pragma unroll
        for (int k = 0; k < D; ++k) F[1 + k] = w[1 + k] * vm;
        F[1 + m] = F[1 + m] + pr * p.inv_eps2;
        F[D + 1] = (w[D + 1] + pr) * vm;
    }
    template <class S, class T> HD static void flux_all(const S* w, S (*F)[NV], const EqParams<T>& p) {
        S irho = jrecip(w[0]);
        S pr = pressure(w, irho, p);
        S pe = pr * p.inv_eps2;
        S Ep = w[D + 1] + pr;
#pragma unroll
        for (int m = 0; m < D; ++m) {
            S vm = w[1 + m] * irho;
            F[m][0] = w[1 + m];
#pragma unroll
            for (int k = 0; k < D; ++k) F[m][1 + k] = w[1 + k] * vm;
            F[m][1 + m] = F[m][1 + m] + pe;
            F[m][D + 1] = Ep * vm;
        }
    }
    template <class S, class T> HD static S wave_speed(const S* w, int m, const EqParams<T>& p) {
        S irho = jrecip(w[0]);
        S pr = pressure(w, irho, p);
        S c = jsqrt(pr * irho * p.gamma);
        return jabs(w[1 + m] * irho) + c * p.inv_eps;
    }
};

// Navier-Stokes (Sec. 5.1, Eq. NavierStokes): the Euler flux minus the viscous flux
// F^v_m = (0, tau_{.m}, tau_{.m}.v + kappa dT/dx_m), tau = mu (grad v + grad v^T - 2/3 div v I),
// which depends on the gradients d[k][j] = d g_k / dx_j of g = (v_1..v_D, T), T = p / (rho R);
// the operator kernel owns the BR2 lifting that provides d.
template <int D> struct NavierStokesEq : EulerEq<D> {
    static constexpr bool NS = true;
    static constexpr int NG = D + 1;
    template <class S, class T> HD static void grad_vars(const S* w, S* g, const EqParams<T>& p) {
        S irho = jrecip(w[0]);
#pragma unroll
        for (int k = 0; k < D; ++k) g[k] = w[1 + k] * irho;
        g[D] = EulerEq<D>::pressure(w, irho, p) * irho * p.gam_eps2;
    }
    template <class S, class T>
    HD static void viscous_flux(const S* w, const S (*d)[D], int m, S* F, const EqParams<T>& p) {
        S irho = jrecip(w[0]);
        S div = d[0][0];
#pragma unroll
        for (int k = 1; k < D; ++k) div = div + d[k][k];
        S energy = d[D][m] * p.kappa;
        F[0] = jconst<S, T>(T(0));
#pragma unroll
        for (int i = 0; i < D; ++i) {
            S t = (d[i][m] + d[m][i]) * p.mu;
            if (i == m) t = t - div * (T(2) / T(3) * p.mu);
            F[1 + i] = t;
            energy = energy + t * (w[1 + i] * irho);
        }
        F[D + 1] = energy;
    }
};

template <class EQ, class S, class T>
HD void numerical_flux(const S* wL, const S* wR, int m, S* f, const EqParams<T>& p) {
    constexpr int NV = EQ::NV;
    S FL[NV], FR[NV];
    EQ::flux_dir(wL, m, FL, p);
    EQ::flux_dir(wR, m, FR, p);
    if (p.flux == FLUX_RUSANOV) {
        S lam = jmax(EQ::wave_speed(wL, m, p), EQ::wave_speed(wR, m, p)) * T(0.5);
#pragma unroll
        for (int v = 0; v < NV; ++v) f[v] = (FL[v] + FR[v]) * T(0.5) + lam * (wL[v] - wR[v]);
    } else if (p.flux == FLUX_LF_LITERAL) {
#pragma unroll
        for (int v = 0; v < NV; ++v)
            f[v] = (FL[v] + FR[v]) * T(0.5) + (wL[v] - wR[v]) * ((v == 0 || v == NV - 1) ? p.inv_eps : T(1));
    } else {
        T lam = p.flux == FLUX_UPWIND ? jabs(p.adv[m]) : (p.flux == FLUX_LF ? p.lam : T(0));
        lam *= T(0.5);
#pragma unroll
        for (int v = 0; v < NV; ++v) f[v] = (FL[v] + FR[v]) * T(0.5) + (wL[v] - wR[v]) * lam;
    }
}
