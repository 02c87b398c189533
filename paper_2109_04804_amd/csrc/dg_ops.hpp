// DGSEM operator kernels for uniform periodic Cartesian meshes (Sec. 3.1).
//
// R1_node = DG[F] := -sum_m (2/h_m) [ sum_lam Dhat[i_m][lam] F_m(node i_m -> lam)
//                                     + lhat_{i_m}(+1) f*_{+m} - lhat_{i_m}(-1) f*_{-m} ]
// (Eq. DGSEM_wt with Cartesian metric terms).  Every operator of the hot path
// is DG[.] applied to a linear combination of the components of a jet-valued
// flux, evaluated once per node and once per face point:
//   R1    jet = w                          DG[F]
//   R2    jet = w + e sigma                DG[F.b]                    (Eq. DGSEM_wtt)
//   RES   jet = w + e sigma                G1 = w - b + DG[-a1dt F.a + bc F.b], G2 = sigma - DG[F.a]
//   JVP   jet = w + e_s sigma + e_d dw + e_e dsigma
//                                          Jw = dw + DG[-a1dt F.d + bc (F.e + F.sd)], Js = dsigma - DG[F.d]
//   KCOL  jet = w + e unit_col   (local)   column col of K = dR1_i/dw_i
//   PCPRE jet = w + e1 vs + e2 (vw - a1dt vs) (local)
//                                          a = vw - bc K vs, c = vs + K (vw - a1dt vs)
// "local": every quantity read from a neighbour is held at its value (the
// direction parts of neighbour traces are zero) -- the element-local Jacobian
// of the BJ_ext preconditioner (Sec. 3.2.3).
//
// Layout: fields x[e][v][node]; traces tr[e][face][v][fp], face = 2m + side
// (side 1 = +e_m), fp enumerates the other directions in increasing order.
// One thread per node; EPB elements per block, staged in LDS.
#pragma once
#include "equations.hpp"

constexpr int ipow(int b, int e) { return e == 0 ? 1 : b * ipow(b, e - 1); }

template <typename T, int NP> struct Basis {
    T Dhat[NP][NP];
    T lp[NP], lm[NP];     // l_i(+1), l_i(-1)
    T lhp[NP], lhm[NP];   // l_i(+-1) / omega_i
};

template <typename T> struct OpArgs {
    const T* fld[4];      // global inputs (meaning per op)
    const T* trc[4];      // neighbour traces of the jet fields (nullptr = zero)
    const T* q[4][3];     // BR1: lifted gradient of jet field j, direction m
    const T* qtr[4];      // BR1: traces of q (face 2m+s holds q_m)
    T* out[2];
    T c0, c1;             // a1dt, bcoef
    int col;              // KCOL: local column
    int nE;               // elements in the mesh (neighbour indexing)
    int e_begin, e_end;   // elements processed by this launch
    int nel[3];
    T two_h[3];
};

// ----------------------------------------------------------------- geometry
template <int D> HD int nbr_elem(int e, int m, int dir, const int* nel) {
    int ex = e % nel[0];
    int ey = D > 1 ? (e / nel[0]) % nel[1] : 0;
    int ez = D > 2 ? e / (nel[0] * nel[1]) : 0;
    if (m == 0) ex = (ex + dir + nel[0]) % nel[0];
    else if (m == 1) ey = (ey + dir + nel[1]) % nel[1];
    else ez = (ez + dir + nel[2]) % nel[2];
    return ex + nel[0] * (ey + (D > 1 ? nel[1] : 1) * ez);
}
// node index of the point with index `i` along direction m through face point fp
template <int D, int NP> HD int node_on_line(int fp, int m, int i) {
    if (D == 1) return i;
    if (D == 2) return m == 0 ? i + NP * fp : fp + NP * i;
    // D == 3: fp = a + NP b over the two other directions in increasing order
    int a = fp % NP, b = fp / NP;
    if (m == 0) return i + NP * (a + NP * b);
    if (m == 1) return a + NP * (i + NP * b);
    return a + NP * (b + NP * i);
}
template <int D, int NP> HD int fp_of_node(int node, int m) {
    if (D == 1) return 0;
    int i = node % NP, j = (node / NP) % NP, k = node / (NP * NP);
    if (D == 2) return m == 0 ? j : i;
    if (m == 0) return j + NP * k;
    if (m == 1) return i + NP * k;
    return i + NP * j;
}

// ----------------------------------------------------------------- op policies
template <typename T> struct OpR1 {
    using S = T;
    static constexpr int NJ = 1, NC = 1;
    static constexpr bool LOCAL = false;
    HD static T load(const OpArgs<T>& a, int j, size_t g, int loc) { return a.fld[0][g]; }
    HD static S make(const T* x, const OpArgs<T>& a) { return x[0]; }
    HD static void combo(const S& f, T* c, const OpArgs<T>& a) { c[0] = f; }
    HD static void output(const OpArgs<T>& a, size_t g, int e, int loc, const T* gv) { a.out[0][g] = gv[0]; }
};

template <typename T> struct OpR2 {
    using S = Dual<T>;
    static constexpr int NJ = 2, NC = 1;
    static constexpr bool LOCAL = false;
    HD static T load(const OpArgs<T>& a, int j, size_t g, int loc) { return a.fld[j][g]; }
    HD static S make(const T* x, const OpArgs<T>& a) { return {x[0], x[1]}; }
    HD static void combo(const S& f, T* c, const OpArgs<T>& a) { c[0] = f.b; }
    HD static void output(const OpArgs<T>& a, size_t g, int e, int loc, const T* gv) { a.out[0][g] = gv[0]; }
};

template <typename T> struct OpRes {   // fld: w, sigma, b
    using S = Dual<T>;
    static constexpr int NJ = 2, NC = 2;
    static constexpr bool LOCAL = false;
    HD static T load(const OpArgs<T>& a, int j, size_t g, int loc) { return a.fld[j][g]; }
    HD static S make(const T* x, const OpArgs<T>& a) { return {x[0], x[1]}; }
    HD static void combo(const S& f, T* c, const OpArgs<T>& a) {
        c[0] = -a.c0 * f.a + a.c1 * f.b;
        c[1] = f.a;
    }
    HD static void output(const OpArgs<T>& a, size_t g, int e, int loc, const T* gv) {
        a.out[0][g] = a.fld[0][g] - a.fld[2][g] + gv[0];
        a.out[1][g] = a.fld[1][g] - gv[1];
    }
};

template <typename T, bool HESS> struct OpJvp {   // fld: w, sigma, dw, dsigma
    using S = Jet5<T>;
    static constexpr int NJ = 4, NC = 2;
    static constexpr bool LOCAL = false;
    HD static T load(const OpArgs<T>& a, int j, size_t g, int loc) { return a.fld[j][g]; }
    HD static S make(const T* x, const OpArgs<T>& a) { return {x[0], x[1], x[2], x[3], T(0)}; }
    HD static void combo(const S& f, T* c, const OpArgs<T>& a) {
        c[0] = -a.c0 * f.d + a.c1 * (HESS ? f.e + f.sd : f.e);
        c[1] = f.d;
    }
    HD static void output(const OpArgs<T>& a, size_t g, int e, int loc, const T* gv) {
        a.out[0][g] = a.fld[2][g] + gv[0];
        a.out[1][g] = a.fld[3][g] - gv[1];
    }
};

template <typename T, int NE> struct OpKcol {   // fld: w; writes K^T[e][col][row] (column-major K)
    using S = Dual<T>;
    static constexpr int NJ = 2, NC = 1;
    static constexpr bool LOCAL = true;
    HD static T load(const OpArgs<T>& a, int j, size_t g, int loc) {
        return j == 0 ? a.fld[0][g] : (loc == a.col ? T(1) : T(0));
    }
    HD static S make(const T* x, const OpArgs<T>& a) { return {x[0], x[1]}; }
    HD static void combo(const S& f, T* c, const OpArgs<T>& a) { c[0] = f.b; }
    HD static void output(const OpArgs<T>& a, size_t g, int e, int loc, const T* gv) {
        a.out[0][((size_t)(e - a.e_begin) * NE + a.col) * NE + loc] = gv[0];
    }
};

template <typename T> struct OpPcPre {   // fld: w, vw, vs
    using S = Dual2<T>;
    static constexpr int NJ = 3, NC = 2;
    static constexpr bool LOCAL = true;
    HD static T load(const OpArgs<T>& a, int j, size_t g, int loc) {
        if (j == 0) return a.fld[0][g];
        if (j == 1) return a.fld[2][g];
        return a.fld[1][g] - a.c0 * a.fld[2][g];
    }
    HD static S make(const T* x, const OpArgs<T>& a) { return {x[0], x[1], x[2]}; }
    HD static void combo(const S& f, T* c, const OpArgs<T>& a) { c[0] = f.b; c[1] = f.c; }
    HD static void output(const OpArgs<T>& a, size_t g, int e, int loc, const T* gv) {
        a.out[0][g] = a.fld[1][g] - a.c1 * gv[0];
        a.out[1][g] = a.fld[2][g] + gv[1];
    }
};

// elements per block: as many as fit 256 threads and ~64 KB of LDS
template <int D, int NP, int NV, int NJ, int NC, typename T> constexpr int op_epb() {
    constexpr int NN = ipow(NP, D), NFP = ipow(NP, D - 1);
    constexpr int bytes = (NJ * NV * NN + NC * D * NV * NN + NC * 2 * D * NV * NFP) * (int)sizeof(T);
    constexpr int by_lds = 65536 / bytes;
    constexpr int by_thr = 256 / NN;
    constexpr int e = by_lds < by_thr ? by_lds : by_thr;
    return e < 1 ? 1 : e;
}

// ----------------------------------------------------------------- trace kernel
template <int D, int NP, int NV, typename T>
__global__ void __launch_bounds__(256) trace_kernel(const T* __restrict__ x, T* __restrict__ tr, int nE,
                                                     Basis<T, NP> bs) {
    constexpr int NN = ipow(NP, D), NFP = ipow(NP, D - 1);
    constexpr int EPB = 256 / NN > 0 ? 256 / NN : 1;
    constexpr int NT = EPB * NN;
    constexpr int PER_E = 2 * D * NV * NFP;
    __shared__ T s[EPB * NV * NN];
    const int tid = threadIdx.x;
    const int e0 = blockIdx.x * EPB;
    const int nloc = min(EPB, nE - e0);
    const size_t base = (size_t)e0 * NV * NN;
    for (int i = tid; i < nloc * NV * NN; i += NT) s[i] = x[base + i];
    __syncthreads();
    for (int i = tid; i < nloc * PER_E; i += NT) {
        int el = i / PER_E, r = i % PER_E;
        int face = r / (NV * NFP), r2 = r % (NV * NFP);
        int v = r2 / NFP, fp = r2 % NFP;
        int m = face >> 1;
        const T* l = (face & 1) ? bs.lp : bs.lm;
        const T* src = s + (el * NV + v) * NN;
        T acc = T(0);
#pragma unroll
        for (int q = 0; q < NP; ++q) acc += l[q] * src[node_on_line<D, NP>(fp, m, q)];
        tr[(size_t)(e0 + el) * PER_E + r] = acc;
    }
}

// ----------------------------------------------------------------- operator kernel
template <int D, int NP, class EQ, class OP, typename T>
__global__ void __launch_bounds__(256) dg_op_kernel(OpArgs<T> a, Basis<T, NP> bs, EqParams<T> ep) {
    constexpr int NN = ipow(NP, D), NFP = ipow(NP, D - 1);
    constexpr int NV = EQ::NV, NJ = OP::NJ, NC = OP::NC;
    constexpr int EPB = op_epb<D, NP, NV, NJ, NC, T>();
    constexpr int NT = EPB * NN;
    using S = typename OP::S;

    __shared__ T s_fld[NJ][EPB][NV][NN];
    __shared__ T s_flx[NC][D][EPB][NV][NN];
    __shared__ T s_fs[NC][EPB][2 * D][NV][NFP];

    const int tid = threadIdx.x;
    const int e0 = a.e_begin + blockIdx.x * EPB;
    const int nloc = min(EPB, a.e_end - e0);

    // 1) stage the jet fields of EPB consecutive elements (contiguous in memory)
    for (int i = tid; i < nloc * NV * NN; i += NT) {
        int el = i / (NV * NN), loc = i % (NV * NN);
        size_t g = (size_t)e0 * NV * NN + i;
#pragma unroll
        for (int j = 0; j < NJ; ++j) (&s_fld[j][0][0][0])[i] = OP::load(a, j, g, loc);
        (void)el;
    }
    __syncthreads();

    const int el = tid / NN, node = tid % NN;
    const bool valid = el < nloc;

    // 2) jet-valued volume fluxes at this node
    if (valid) {
        S wn[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            T x[NJ];
#pragma unroll
            for (int j = 0; j < NJ; ++j) x[j] = s_fld[j][el][v][node];
            wn[v] = OP::make(x, a);
        }
        S F[D][NV];
        EQ::flux_all(wn, F, ep);
#pragma unroll
        for (int m = 0; m < D; ++m)
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                T c[NC];
                OP::combo(F[m][v], c, a);
#pragma unroll
                for (int k = 0; k < NC; ++k) s_flx[k][m][el][v][node] = c[k];
            }
    }

    // 3) numerical fluxes at the face points (own trace from LDS, neighbour trace from HBM)
    for (int i = tid; i < nloc * 2 * D * NFP; i += NT) {
        int fel = i / (2 * D * NFP), r = i % (2 * D * NFP);
        int face = r / NFP, fp = r % NFP;
        int m = face >> 1, side = face & 1;
        int fe = e0 + fel;
        const T* l = side ? bs.lp : bs.lm;
        S own[NV], nb[NV];
        int enb = nbr_elem<D>(fe, m, side ? 1 : -1, a.nel);
        size_t nbase = ((size_t)enb * 2 * D + (2 * m + 1 - side)) * NV * NFP + fp;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            T x[NJ], y[NJ];
#pragma unroll
            for (int j = 0; j < NJ; ++j) {
                T acc = T(0);
#pragma unroll
                for (int q = 0; q < NP; ++q) acc += l[q] * s_fld[j][fel][v][node_on_line<D, NP>(fp, m, q)];
                x[j] = acc;
                const T* t = (OP::LOCAL && j > 0) ? nullptr : a.trc[j];
                y[j] = t ? t[nbase + (size_t)v * NFP] : T(0);
            }
            own[v] = OP::make(x, a);
            nb[v] = OP::make(y, a);
        }
        S f[NV];
        if (side) numerical_flux<EQ>(own, nb, m, f, ep);
        else numerical_flux<EQ>(nb, own, m, f, ep);
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            T c[NC];
            OP::combo(f[v], c, a);
#pragma unroll
            for (int k = 0; k < NC; ++k) s_fs[k][fel][face][v][fp] = c[k];
        }
    }
    __syncthreads();
    if (!valid) return;

    // 4) volume sweep + surface lifting, DG[.] per combination and variable
    int idx[3] = {node % NP, (node / NP) % NP, node / (NP * NP)};
    T gv[NC];
    const int e = e0 + el;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
#pragma unroll
        for (int k = 0; k < NC; ++k) {
            T acc = T(0);
#pragma unroll
            for (int m = 0; m < D; ++m) {
                const int im = idx[m];
                const int stride = m == 0 ? 1 : (m == 1 ? NP : NP * NP);
                const int b0 = node - im * stride;
                T s = T(0);
#pragma unroll
                for (int q = 0; q < NP; ++q) s += bs.Dhat[im][q] * s_flx[k][m][el][v][b0 + q * stride];
                const int fp = fp_of_node<D, NP>(node, m);
                s += bs.lhp[im] * s_fs[k][el][2 * m + 1][v][fp] - bs.lhm[im] * s_fs[k][el][2 * m][v][fp];
                acc += a.two_h[m] * s;
            }
            gv[k] = -acc;
        }
        const int loc = v * NN + node;
        OP::output(a, (size_t)e * NV * NN + loc, e, loc, gv);
    }
}
