// Host-side launch of the DGSEM operator kernels for one (equation, d) family.
#pragma once
#include <hip/hip_runtime.h>
#include "dg_ops.hpp"

enum {
    OPK_TRACE = 0, OPK_R1, OPK_R2, OPK_RES, OPK_JVP, OPK_JVP_NOHESS, OPK_KCOL, OPK_PCPRE,
    OPK_LIFT,     // BR1 lifting (viscous Burgers only)
    OPK_LINLOC,   // x + c0 K(w) s, K the element-local Jacobian of BJ_ext
    OPK_KHCOL     // columns of K and of the element-local Hessian block H (BJ^H_ext, FP64)
};

struct GeomHost {
    int D, NP, NV, nE;
    int nel[3];
    double two_h[3];
    const double* basis64;   // device copies of the 1-D operators (dg_ops.hpp layout)
    const float* basis32;
    double adv[3], lam, nu, gamma, eps;
    double mu, kappa, gam_eps2, eta;   // Navier-Stokes: viscosity, heat conductivity, 1/R, BR2 eta
    int flux;
};

struct LaunchReq {
    int op;
    const void* fld[4];
    const void* trc[4];
    const void* q[4][3];
    const void* qtr[4];
    void* out[4];
    void* nsg[4];         // BR2: viscous fluxes at the face points per jet component (Navier-Stokes)
    int aux;              // 1: run the BR2 face-gradient kernel of this op instead of the op
    double c0, c1;
    int col;
    int e_begin, e_end;   // element range (e_end <= 0: whole mesh)
    hipStream_t stream;
    const LaunchReq* pair;   // the same op on a second system's arrays in the same launch (or null)
};

template <typename T> const T* basis_ptr(const GeomHost& g);
template <> inline const double* basis_ptr<double>(const GeomHost& g) { return g.basis64; }
template <> inline const float* basis_ptr<float>(const GeomHost& g) { return g.basis32; }

template <typename T> EqParams<T> make_eq(const GeomHost& g) {
    EqParams<T> p;
    for (int m = 0; m < 3; ++m) p.adv[m] = (T)g.adv[m];
    p.lam = (T)g.lam;
    p.nu = (T)g.nu;
    p.gm1 = (T)(g.gamma - 1.0);
    p.gamma = (T)g.gamma;
    p.half_eps2 = (T)(0.5 * g.eps * g.eps);
    p.inv_eps = (T)(1.0 / g.eps);
    p.inv_eps2 = (T)(1.0 / (g.eps * g.eps));
    p.mu = (T)g.mu;
    p.kappa = (T)g.kappa;
    p.gam_eps2 = (T)g.gam_eps2;
    p.eta = (T)g.eta;
    p.flux = g.flux;
    return p;
}

template <typename T> OpArgs<T> make_args(const GeomHost& g, const LaunchReq& r) {
    OpArgs<T> a;
    for (int j = 0; j < 4; ++j) {
        a.fld[j] = (const T*)r.fld[j];
        a.trc[j] = (const T*)r.trc[j];
        a.qtr[j] = (const T*)r.qtr[j];
        a.nsg[j] = (T*)r.nsg[j];
        for (int m = 0; m < 3; ++m) a.q[j][m] = (const T*)r.q[j][m];
    }
    a.out[0] = (T*)r.out[0];
    a.out[1] = (T*)r.out[1];
    a.basis = basis_ptr<T>(g);
    a.c0 = (T)r.c0;
    a.c1 = (T)r.c1;
    a.col = r.col;
    a.nE = g.nE;
    a.e_begin = r.e_end > 0 ? r.e_begin : 0;
    a.e_end = r.e_end > 0 ? r.e_end : g.nE;
    for (int m = 0; m < 3; ++m) {
        a.nel[m] = g.nel[m];
        a.two_h[m] = (T)g.two_h[m];
    }
    return a;
}

// BR2 face gradients of the jet of OP over the whole mesh (Navier-Stokes only)
template <int D, int NP, class EQ, class OP, typename T>
hipError_t launch_nsaux(const GeomHost& g, const LaunchReq& r) {
    if constexpr (!EQ::NS) {
        return hipErrorInvalidValue;
    } else {
        constexpr int NN = ipow(NP, D);
        constexpr int EPB = aux_epb<D, NP, EQ, OP, T>();
        OpArgs<T> a = make_args<T>(g, r);
        int grid = (g.nE + EPB - 1) / EPB;
        if (grid <= 0) return hipSuccess;
        hipLaunchKernelGGL((ns_facegrad_kernel<D, NP, EQ, OP, T>), dim3(grid), dim3(EPB * NN), 0, r.stream, a,
                           make_eq<T>(g));
        return hipGetLastError();
    }
}

template <int D, int NP, class EQ, class OP, typename T>
hipError_t launch_op(const GeomHost& g, const LaunchReq& r) {
    if (r.aux) return launch_nsaux<D, NP, EQ, OP, T>(g, r);
    constexpr int NN = ipow(NP, D);
    constexpr int EPB = kernel_epb<D, NP, EQ, OP, T>();
    OpArgs<T> a = make_args<T>(g, r);
    int grid = (a.e_end - a.e_begin + EPB - 1) / EPB;
    if (grid <= 0) return hipSuccess;
    OpArgs<T> a1 = r.pair ? make_args<T>(g, *r.pair) : a;
    const int grid1 = r.pair ? (a1.e_end - a1.e_begin + EPB - 1) / EPB : 0;
    dim3 gd(grid + grid1, (r.op == OPK_KCOL || r.op == OPK_KHCOL) ? EQ::NV * NN : 1);   // one grid row per column
    hipLaunchKernelGGL((dg_op_kernel<D, NP, EQ, OP, T>), gd, dim3(EPB * NN), 0, r.stream, a, make_eq<T>(g), a1,
                       grid);
    return hipGetLastError();
}

template <int D, int NP, class EQ, typename T> hipError_t launch_family_np(const GeomHost& g, const LaunchReq& r) {
    constexpr int NV = EQ::NV;
    constexpr int NN = ipow(NP, D);
    switch (r.op) {
    case OPK_TRACE: {
        constexpr int EPB = trace_epb<NN>();
        int grid = (g.nE + EPB - 1) / EPB;
        if (grid == 0) return hipSuccess;
        const int nf = r.col > 1 ? r.col : 1;   // consecutive fields (col = their number)
        const T* x2 = r.pair ? (const T*)r.pair->fld[0] : (const T*)r.fld[0];
        T* tr2 = r.pair ? (T*)r.pair->out[0] : (T*)r.out[0];
        hipLaunchKernelGGL((trace_kernel<D, NP, NV, T>), dim3(grid, nf, r.pair ? 2 : 1), dim3(trace_threads<NN>()), 0,
                           r.stream,
                           (const T*)r.fld[0], (T*)r.out[0], g.nE, basis_ptr<T>(g), x2, tr2);
        return hipGetLastError();
    }
    case OPK_R1: return launch_op<D, NP, EQ, OpR1<T>, T>(g, r);
    case OPK_R2: return launch_op<D, NP, EQ, OpR2<T>, T>(g, r);
    case OPK_RES: return launch_op<D, NP, EQ, OpRes<T>, T>(g, r);
    case OPK_JVP: return launch_op<D, NP, EQ, OpJvp<T, true>, T>(g, r);
    case OPK_JVP_NOHESS: return launch_op<D, NP, EQ, OpJvp<T, false>, T>(g, r);
    case OPK_KCOL: return launch_op<D, NP, EQ, OpKcol<T, NV * NN>, T>(g, r);
    case OPK_PCPRE: return launch_op<D, NP, EQ, OpPcPre<T>, T>(g, r);
    case OPK_LINLOC: return launch_op<D, NP, EQ, OpLin<T, true>, T>(g, r);
    case OPK_KHCOL:
        if constexpr (sizeof(T) == 8) return launch_op<D, NP, EQ, OpKHcol<T, NV * NN>, T>(g, r);
        return hipErrorInvalidValue;
    case OPK_LIFT: {
        if (!EQ::VISC) return hipErrorInvalidValue;
        constexpr int EPB = 256 / NN > 0 ? 256 / NN : 1;
        int grid = (g.nE + EPB - 1) / EPB;
        if (grid == 0) return hipSuccess;
        hipLaunchKernelGGL((lift_trace_kernel<D, NP, T>), dim3(grid), dim3(EPB * NN), 0, r.stream,
                           (const T*)r.fld[0], (const T*)r.trc[0], (T*)r.out[0], make_args<T>(g, r));
        return hipGetLastError();
    }
    default: return hipErrorInvalidValue;
    }
}

// largest N + 1 instantiated: 8 (N = 7) in 1-D and 2-D, 6 in 3-D (a 3-D element of 343 nodes exceeds
// one 256-thread block with one thread per node); with the BR2 lifting in 3-D 5, where the LDS of
// the lifted gradients in hyper-dual FP64 still fits gfx950's 160 KB per workgroup
template <int D, class EQ> constexpr int max_np() {
    if constexpr (D == 3 && EQ::NS) return 5;
    else if constexpr (D == 3) return 6;
    else return 8;
}

template <int D, class EQ> hipError_t launch_family(const GeomHost& g, const LaunchReq& r, int f32) {
#define HBPC_NP_CASE(NPV)                                                                  \
    case NPV:                                                                              \
        if constexpr (NPV <= max_np<D, EQ>())                                              \
            return f32 ? launch_family_np<D, NPV, EQ, float>(g, r)                         \
                       : launch_family_np<D, NPV, EQ, double>(g, r);                       \
        return hipErrorInvalidValue;
    switch (g.NP) {
        HBPC_NP_CASE(3)
        HBPC_NP_CASE(4)
        HBPC_NP_CASE(5)
        HBPC_NP_CASE(6)
        HBPC_NP_CASE(7)
        HBPC_NP_CASE(8)
    default: return hipErrorInvalidValue;
    }
#undef HBPC_NP_CASE
}
