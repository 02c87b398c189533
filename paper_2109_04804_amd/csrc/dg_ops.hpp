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
//   JVP   jet = w + e_s sigma + e_d dw + e_s e_d dsigma   (hyper-dual; without the Hessian term:
//               w + e1 dw + e2 dsigma)
//                                          Jw = dw + DG[-a1dt F.d + bc F.m], Js = dsigma - DG[F.d]
//               (F.m = F'(w) dsigma + F''(w)[sigma, dw]; without the Hessian term F'(w) dsigma)
//   KCOL  jet = w + e unit_col   (local)   column col of K = dR1_i/dw_i
//   KHCOL jet = w + e_s sigma + e_d unit_col (local in e_d)
//                                          column col of K and of H = dR2_i/dw_i (BJ^H_ext)
//   PCPRE jet = w + e1 vs + e2 (vw - a1dt vs) (local)
//                                          a = vw - bc K vs, c = vs + K (vw - a1dt vs)
// "local": every quantity read from a neighbour is held at its value (the
// direction parts of neighbour traces are zero) -- the element-local Jacobian
// of the BJ_ext preconditioner (Sec. 3.2.3).  Each op names NGLOB: jet fields
// j < NGLOB read their neighbour traces, the others are zero across faces.
//
// Layout: fields x[e][v][node]; traces tr[e][face][v][fp], face = 2m + side
// (side 1 = +e_m), fp enumerates the other directions in increasing order.
// One thread per node; EPB elements per block, staged in LDS.
#pragma once
#include "equations.hpp"

constexpr int ipow(int b, int e) { return e == 0 ? 1 : b * ipow(b, e - 1); }

// 1-D operators in device memory, copied to LDS by every block:
//   Dhat[NP*NP] (Dhat[i*NP+lam]), lp[NP] = l_i(+1), lm[NP] = l_i(-1),
//   lhp[NP] = l_i(+1)/omega_i, lhm[NP] = l_i(-1)/omega_i,
//   for the BR2 lifting: Dstr[NP*NP] (Dstr[i*NP+lam] = l_lam'(xi_i)), lDp[NP], lDm[NP]
//   (lDp[lam] = sum_i l_i(+1) Dstr[i][lam]), c[2] = sum_i l_i(+-1)^2 / omega_i
template <int NP> constexpr int basis_len() { return 2 * NP * NP + 6 * NP + 2; }
template <int NP> struct BOff {
    static constexpr int D = 0, LP = NP * NP, LM = LP + NP, LHP = LM + NP, LHM = LHP + NP;
    static constexpr int DS = LHM + NP, LDP = DS + NP * NP, LDM = LDP + NP, CP = LDM + NP, CM = CP + 1;
};

template <typename T> struct OpArgs {
    const T* fld[4];      // global inputs (meaning per op)
    const T* trc[4];      // neighbour traces of the jet fields (nullptr = zero)
    const T* q[4][3];     // BR1: lifted gradient of jet field j, direction m
    const T* qtr[4];      // BR1: traces of q (face 2m+s holds q_m)
    T* nsg[4];            // BR2 face gradients of jet component j (written by the face-gradient
                          // kernel, read as neighbour data by the operator kernel)
    T* out[2];
    const T* basis;       // 1-D operators (layout above)
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
    static constexpr int NGLOB = NJ;
    HD static T load(const OpArgs<T>& a, int j, size_t g, int loc) { return a.fld[0][g]; }
    HD static S make(const T* x, const OpArgs<T>& a) { return x[0]; }
    HD static void split(const S& v, T* x) { jet_split(v, x); }
    HD static void combo(const S& f, T* c, const OpArgs<T>& a) { c[0] = f; }
    HD static void output(const OpArgs<T>& a, size_t g, int e, int loc, const T* gv) { a.out[0][g] = gv[0]; }
};

template <typename T> struct OpR2 {
    using S = Dual<T>;
    static constexpr int NJ = 2, NC = 1;
    static constexpr int NGLOB = NJ;
    HD static T load(const OpArgs<T>& a, int j, size_t g, int loc) { return a.fld[j][g]; }
    HD static S make(const T* x, const OpArgs<T>& a) { return {x[0], x[1]}; }
    HD static void split(const S& v, T* x) { jet_split(v, x); }
    HD static void combo(const S& f, T* c, const OpArgs<T>& a) { c[0] = f.b; }
    HD static void output(const OpArgs<T>& a, size_t g, int e, int loc, const T* gv) { a.out[0][g] = gv[0]; }
};

template <typename T> struct OpRes {   // fld: w, sigma, b
    using S = Dual<T>;
    static constexpr int NJ = 2, NC = 2;
    static constexpr int NGLOB = NJ;
    HD static T load(const OpArgs<T>& a, int j, size_t g, int loc) { return a.fld[j][g]; }
    HD static S make(const T* x, const OpArgs<T>& a) { return {x[0], x[1]}; }
    HD static void split(const S& v, T* x) { jet_split(v, x); }
    HD static void combo(const S& f, T* c, const OpArgs<T>& a) {
        c[0] = -a.c0 * f.a + a.c1 * f.b;
        c[1] = f.a;
    }
    HD static void output(const OpArgs<T>& a, size_t g, int e, int loc, const T* gv) {
        a.out[0][g] = a.fld[0][g] - a.fld[2][g] + gv[0];
        a.out[1][g] = a.fld[1][g] - gv[1];
    }
};

template <typename T, bool HESS> struct JvpJet;
template <typename T> struct JvpJet<T, true> {   // w + e_s sigma + e_d dw + e_s e_d dsigma
    using S = HDual<T>;
    HD static S make(const T* x) { return {x[0], x[1], x[2], x[3]}; }
    HD static void split(const S& v, T* x) { jet_split(v, x); }
    HD static T first(const S& f) { return f.d; }
    HD static T second(const S& f) { return f.m; }
};
template <typename T> struct JvpJet<T, false> {   // w + e1 dw + e2 dsigma
    using S = Dual2<T>;
    HD static S make(const T* x) { return {x[0], x[2], x[3]}; }
    HD static void split(const S& v, T* x) { x[0] = v.a; x[1] = T(0); x[2] = v.b; x[3] = v.c; }
    HD static T first(const S& f) { return f.b; }
    HD static T second(const S& f) { return f.c; }
};

template <typename T, bool HESS> struct OpJvp {   // fld: w, sigma, dw, dsigma
    using J = JvpJet<T, HESS>;
    using S = typename J::S;
    static constexpr int NJ = 4, NC = 2;
    static constexpr int NGLOB = NJ;
    HD static T load(const OpArgs<T>& a, int j, size_t g, int loc) { return a.fld[j][g]; }
    HD static S make(const T* x, const OpArgs<T>& a) { return J::make(x); }
    HD static void split(const S& v, T* x) { J::split(v, x); }
    HD static void combo(const S& f, T* c, const OpArgs<T>& a) {
        c[0] = -a.c0 * J::first(f) + a.c1 * J::second(f);
        c[1] = J::first(f);
    }
    HD static void output(const OpArgs<T>& a, size_t g, int e, int loc, const T* gv) {
        a.out[0][g] = a.fld[2][g] + gv[0];
        a.out[1][g] = a.fld[3][g] - gv[1];
    }
};

template <typename T, int NE> struct OpKcol {   // fld: w; column = blockIdx.y; writes K^T[e][col][row]
    using S = Dual<T>;
    static constexpr int NJ = 2, NC = 1;
    static constexpr int NGLOB = 1;
    HD static T load(const OpArgs<T>& a, int j, size_t g, int loc) {
        return j == 0 ? a.fld[0][g] : (loc == (int)blockIdx.y ? T(1) : T(0));
    }
    HD static S make(const T* x, const OpArgs<T>& a) { return {x[0], x[1]}; }
    HD static void split(const S& v, T* x) { jet_split(v, x); }
    HD static void combo(const S& f, T* c, const OpArgs<T>& a) { c[0] = f.b; }
    HD static void output(const OpArgs<T>& a, size_t g, int e, int loc, const T* gv) {
        a.out[0][((size_t)(e - a.e_begin) * NE + blockIdx.y) * NE + loc] = gv[0];
    }
};

// fld: w, sigma; column = blockIdx.y; writes K^T (out[0]) and H^T (out[1]), H = dR2_i/dw_i at
// (w, sigma): the e_s e_d part of the hyper-dual flux is F''(w)[sigma, e_col].  The neighbours'
// sigma enters the face fluxes (NGLOB = 2); their dependence on w does not.
template <typename T, int NE> struct OpKHcol {
    using S = HDual<T>;
    static constexpr int NJ = 4, NC = 2;
    static constexpr int NGLOB = 2;
    HD static T load(const OpArgs<T>& a, int j, size_t g, int loc) {
        if (j < 2) return a.fld[j][g];
        return (j == 2 && loc == (int)blockIdx.y) ? T(1) : T(0);
    }
    HD static S make(const T* x, const OpArgs<T>& a) { return {x[0], x[1], x[2], x[3]}; }
    HD static void split(const S& v, T* x) { jet_split(v, x); }
    HD static void combo(const S& f, T* c, const OpArgs<T>& a) { c[0] = f.d; c[1] = f.m; }
    HD static void output(const OpArgs<T>& a, size_t g, int e, int loc, const T* gv) {
        const size_t i = ((size_t)(e - a.e_begin) * NE + blockIdx.y) * NE + loc;
        a.out[0][i] = gv[0];
        a.out[1][i] = gv[1];
    }
};

template <typename T> struct OpPcPre {   // fld: w, vw, vs
    using S = Dual2<T>;
    static constexpr int NJ = 3, NC = 2;
    static constexpr int NGLOB = 1;
    HD static T load(const OpArgs<T>& a, int j, size_t g, int loc) {
        if (j == 0) return a.fld[0][g];
        if (j == 1) return a.fld[2][g];
        return a.fld[1][g] - a.c0 * a.fld[2][g];
    }
    HD static S make(const T* x, const OpArgs<T>& a) { return {x[0], x[1], x[2]}; }
    HD static void split(const S& v, T* x) { jet_split(v, x); }
    HD static void combo(const S& f, T* c, const OpArgs<T>& a) { c[0] = f.b; c[1] = f.c; }
    HD static void output(const OpArgs<T>& a, size_t g, int e, int loc, const T* gv) {
        a.out[0][g] = a.fld[1][g] - a.c1 * gv[0];
        a.out[1][g] = a.fld[2][g] + gv[1];
    }
};

// fld: w, s, x;  out = x + c0 R1'(w) s, with LOC the neighbour values of s held at zero, i.e.
// the element-local Jacobian K of BJ_ext
template <typename T, bool LOC> struct OpLin {
    using S = Dual<T>;
    static constexpr int NJ = 2, NC = 1;
    static constexpr int NGLOB = LOC ? 1 : NJ;
    HD static T load(const OpArgs<T>& a, int j, size_t g, int loc) { return a.fld[j][g]; }
    HD static S make(const T* x, const OpArgs<T>& a) { return {x[0], x[1]}; }
    HD static void split(const S& v, T* x) { jet_split(v, x); }
    HD static void combo(const S& f, T* c, const OpArgs<T>& a) { c[0] = f.b; }
    HD static void output(const OpArgs<T>& a, size_t g, int e, int loc, const T* gv) {
        a.out[0][g] = a.fld[2][g] + a.c0 * gv[0];
    }
};

// elements per block of the operator kernel: the count (up to 256 threads) that keeps the most
// waves resident on a CU under gfx950's 160 KB of LDS (per CU and per workgroup), counted up to
// 12 waves (3 per SIMD: the register budget of the jet kernels, 100-160 VGPRs, allows no more);
// ties go to more elements per block (fewer idle threads in the face phase).  bytes: LDS per element.
template <int NN> constexpr int best_epb(int bytes, bool small_ties = false) {
    int best = 1, best_w = 0;
    for (int e = 1; e * NN <= 256; ++e) {
        const int blk = e * bytes + 1024;   // + the 1-D operators
        if (blk > 163840) break;
        const int per_cu = 163840 / blk;
        int w = per_cu * ((e * NN + 63) / 64);
        if (w > 12) w = 12;
        if (small_ties ? w > best_w : w >= best_w) {
            best_w = w;
            best = e;
        }
    }
    return best;
}

// Navier-Stokes: number of lifted variables g = (v, T) (0 for the other equations)
template <class EQ> constexpr int eq_ng() {
    if constexpr (EQ::NS) return EQ::NG;
    else return 0;
}
// LDS bytes per element of the BR2 lifting: g at the nodes, the jumps at the face points, the
// strong gradients at the nodes, in the jet type S
template <int D, int NP, class EQ, class S> constexpr int ns_lds_bytes() {
    constexpr int NN = ipow(NP, D), NFP = ipow(NP, D - 1), NG = eq_ng<EQ>();
    return (NG * NN + NG * 2 * D * NFP + NG * D * NN) * (int)sizeof(S);
}
// LDS per element of dg_op_kernel: jet fields, one direction's flux combinations, face-flux
// combinations, BR1 lifted gradients and u* (viscous Burgers), the BR2 lifting (Navier-Stokes)
template <int D, int NP, class EQ, class OP, typename T> constexpr int kernel_epb() {
    constexpr int NN = ipow(NP, D), NFP = ipow(NP, D - 1), NV = EQ::NV;
    constexpr int NQ = EQ::VISC ? OP::NJ : 0;
    constexpr int bytes = (OP::NJ * NV * NN + OP::NC * NV * NN + OP::NC * 2 * D * NV * NFP + NQ * D * NN +
                           NQ * 2 * D * NFP) * (int)sizeof(T) +
                          ns_lds_bytes<D, NP, EQ, typename OP::S>();
    return best_epb<NN>(bytes);
}
// elements per block of the BR2 face-gradient kernel (jet fields and the lifting in LDS)
// (the lifting data leave a CU only a few waves whatever the block size; there independent small
// blocks hide latency better than one block of several waves, and this kernel has no face phase
// whose threads a one-element block would leave idle)
template <int D, int NP, class EQ, class OP, typename T> constexpr int aux_epb() {
    constexpr int NN = ipow(NP, D);
    constexpr int bytes = OP::NJ * EQ::NV * NN * (int)sizeof(T) + ns_lds_bytes<D, NP, EQ, typename OP::S>();
    return best_epb<NN>(bytes, true);
}

// ----------------------------------------------------------------- trace kernel
// threads per block (whole elements' nodes, at most 256) and elements per block (twice as many:
// each thread loads and interpolates for two elements, more loads in flight per block)
template <int NN> constexpr int trace_threads() { return (256 / NN > 0 ? 256 / NN : 1) * NN; }
template <int NN> constexpr int trace_epb() { return 2 * (256 / NN > 0 ? 256 / NN : 1); }

template <int D, int NP, int NV, typename T>
__global__ void __launch_bounds__(256) trace_kernel(const T* x, T* tr, int nE,
                                                     const T* __restrict__ basis, const T* x2, T* tr2) {
    constexpr int NN = ipow(NP, D), NFP = ipow(NP, D - 1);
    constexpr int EPB = trace_epb<NN>();
    constexpr int NT = trace_threads<NN>();
    constexpr int PER_E = 2 * D * NV * NFP;
    __shared__ __align__(16) T s[EPB * NV * NN];
    __shared__ T s_l[2][NP];      // l(-1), l(+1)
    const int tid = threadIdx.x;
    const int e0 = blockIdx.x * EPB;
    const int nloc = min(EPB, nE - e0);
    const size_t base = (size_t)e0 * NV * NN;
    // blockIdx.z = 1: the second system's fields (paired stage solves); field blockIdx.y of
    // consecutive fields (stride: one state vector in, one trace array out)
    if (blockIdx.z) {
        x = x2;
        tr = tr2;
    }
    x += (size_t)blockIdx.y * nE * NV * NN;
    tr += (size_t)blockIdx.y * nE * PER_E;
    if (tid < 2 * NP) s_l[tid / NP][tid % NP] = basis[(tid < NP ? BOff<NP>::LM : BOff<NP>::LP) + tid % NP];
    constexpr int VW = 16 / (int)sizeof(T);   // values per 16-byte load
    if constexpr ((NV * NN) % VW == 0) {
        if ((reinterpret_cast<uintptr_t>(x) & 15) == 0) {   // whole elements are whole 16-byte pieces
            typedef T VT __attribute__((ext_vector_type(VW)));
            const VT* xv = reinterpret_cast<const VT*>(x + base);
            VT* sv = reinterpret_cast<VT*>(s);
            for (int i = tid; i < nloc * NV * NN / VW; i += NT) sv[i] = xv[i];
        } else {
            for (int i = tid; i < nloc * NV * NN; i += NT) s[i] = x[base + i];
        }
    } else {
        for (int i = tid; i < nloc * NV * NN; i += NT) s[i] = x[base + i];
    }
    __syncthreads();
    for (int i = tid; i < nloc * PER_E; i += NT) {
        int el = i / PER_E, r = i % PER_E;
        int face = r / (NV * NFP), r2 = r % (NV * NFP);
        int v = r2 / NFP, fp = r2 % NFP;
        int m = face >> 1;
        const T* l = s_l[face & 1];
        const T* src = s + (el * NV + v) * NN;
        T acc = T(0);
#pragma unroll
        for (int q = 0; q < NP; ++q) acc += l[q] * src[node_on_line<D, NP>(fp, m, q)];
        tr[(size_t)(e0 + el) * PER_E + r] = acc;
    }
}

// ----------------------------------------------------------------- BR1 lift traces
// Traces of the BR1-lifted gradient of a scalar field u (NV = 1):
//   q_m = (2/h_m)[Dhat u + lhat(+1) u*_+ - lhat(-1) u*_-], u* = (u_own + u_nbr)/2,
// qtr[e][2m+side][fp] = sum_i l_i(+-1) q_m(line through fp).  Faces of other
// directions are not written (never read).
template <int D, int NP, typename T>
__global__ void __launch_bounds__(256) lift_trace_kernel(const T* __restrict__ u, const T* __restrict__ tru,
                                                          T* __restrict__ qtr, OpArgs<T> a) {
    constexpr int NN = ipow(NP, D), NFP = ipow(NP, D - 1);
    constexpr int EPB = 256 / NN > 0 ? 256 / NN : 1;
    constexpr int NT = EPB * NN;
    __shared__ T s_u[EPB][NN];
    __shared__ T s_us[EPB][2 * D][NFP];
    __shared__ T s_q[D][EPB][NN];
    __shared__ T s_b[basis_len<NP>()];
    const int tid = threadIdx.x;
    const int e0 = blockIdx.x * EPB;
    const int nloc = min(EPB, a.nE - e0);
    for (int i = tid; i < basis_len<NP>(); i += NT) s_b[i] = a.basis[i];
    for (int i = tid; i < nloc * NN; i += NT) (&s_u[0][0])[i] = u[(size_t)e0 * NN + i];
    __syncthreads();
    for (int i = tid; i < nloc * 2 * D * NFP; i += NT) {
        const int fel = i / (2 * D * NFP), r = i % (2 * D * NFP);
        const int face = r / NFP, fp = r % NFP;
        const int m = face >> 1, side = face & 1;
        const T* l = s_b + (side ? BOff<NP>::LP : BOff<NP>::LM);
        T own = T(0);
        for (int q = 0; q < NP; ++q) own += l[q] * s_u[fel][node_on_line<D, NP>(fp, m, q)];
        const int enb = nbr_elem<D>(e0 + fel, m, side ? 1 : -1, a.nel);
        s_us[fel][face][fp] = T(0.5) * (own + tru[((size_t)enb * 2 * D + (2 * m + 1 - side)) * NFP + fp]);
    }
    __syncthreads();
    const int el = tid / NN, node = tid % NN;
    if (el < nloc) {
        const int id3[3] = {node % NP, (node / NP) % NP, node / (NP * NP)};
#pragma unroll
        for (int m = 0; m < D; ++m) {
            const int im = id3[m];
            const int stride = m == 0 ? 1 : (m == 1 ? NP : NP * NP);
            const int b0 = node - im * stride;
            const T* Drow = s_b + BOff<NP>::D + im * NP;
            T sv = T(0);
            for (int q = 0; q < NP; ++q) sv += Drow[q] * s_u[el][b0 + q * stride];
            const int fpm = fp_of_node<D, NP>(node, m);
            sv += s_b[BOff<NP>::LHP + im] * s_us[el][2 * m + 1][fpm] - s_b[BOff<NP>::LHM + im] * s_us[el][2 * m][fpm];
            s_q[m][el][node] = a.two_h[m] * sv;
        }
    }
    __syncthreads();
    for (int i = tid; i < nloc * 2 * D * NFP; i += NT) {
        const int fel = i / (2 * D * NFP), r = i % (2 * D * NFP);
        const int face = r / NFP, fp = r % NFP;
        const int m = face >> 1, side = face & 1;
        const T* l = s_b + (side ? BOff<NP>::LP : BOff<NP>::LM);
        T acc = T(0);
        for (int q = 0; q < NP; ++q) acc += l[q] * s_q[m][fel][node_on_line<D, NP>(fp, m, q)];
        qtr[((size_t)(e0 + fel) * 2 * D + face) * NFP + fp] = acc;
    }
}

// ----------------------------------------------------------------- BR2 lifting (Navier-Stokes)
// Sec. 5.1 with the lifting in strong form: g = (v_1..v_D, T) at the nodes, g at a face point
// from the trace of w there, the jump J = g* - g_own = (g(w_nbr) - g(w_own))/2 at every face
// point, the strong (broken) gradient (2/h_j) Dstr g_k at the nodes, and
//   volume gradient   d_kj = (2/h_j)[Dstr g_k + lhat(+1) J_k(+e_j) - lhat(-1) J_k(-e_j)]
//   face gradient     d_kj(face +-e_m) = [(2/h_j) Dstr_j g_k](+-1 along m) +- delta_jm eta (2/h_m) c_+- J_k
// (BR2: the broken gradient plus eta times the face's own local lifting, c_+- = sum l(+-1)^2/omega).
// Layouts in LDS (jet type S): s_g[k][el][node], s_jmp[k][el][face][fp], s_dv[k][j][el][node].
// AUX: components j >= NGLOB of the jet are zero (the face-gradient kernel produces only the
// parts that neighbours read).
template <class OP, bool AUX, typename T, int EPB, int NV, int NN>
__device__ __forceinline__ typename OP::S ns_jet(const OpArgs<T>& a, const T (*s_fld)[EPB][NV][NN], int el, int v,
                                                 int node) {
    T x[OP::NJ];
#pragma unroll
    for (int j = 0; j < OP::NJ; ++j) x[j] = (AUX && j >= OP::NGLOB) ? T(0) : s_fld[j][el][v][node];
    return OP::make(x, a);
}

// phase A (every node): g into s_g
template <int D, int NP, class EQ, class OP, bool AUX, typename T, int EPB, int NN>
__device__ __forceinline__ void ns_stage_g(const OpArgs<T>& a, const EqParams<T>& ep,
                                           const T (*s_fld)[EPB][EQ::NV][NN], typename OP::S* s_g, int el,
                                           int node) {
    using S = typename OP::S;
    constexpr int NV = EQ::NV, NG = EQ::NG;
    S wn[NV], g[NG];
#pragma unroll
    for (int v = 0; v < NV; ++v) wn[v] = ns_jet<OP, AUX, T, EPB, NV, NN>(a, s_fld, el, v, node);
    EQ::grad_vars(wn, g, ep);
#pragma unroll
    for (int k = 0; k < NG; ++k) s_g[(k * EPB + el) * NN + node] = g[k];
}

// phase A (every face point): the jump J into s_jmp
template <int D, int NP, class EQ, class OP, bool AUX, typename T, int EPB, int NN, int NFP>
__device__ __forceinline__ void ns_face_jump(const OpArgs<T>& a, const EqParams<T>& ep, const T* s_b,
                                             const T (*s_fld)[EPB][EQ::NV][NN], typename OP::S* s_jmp, int fel,
                                             int fe, int face, int fp) {
    using S = typename OP::S;
    constexpr int NV = EQ::NV, NG = EQ::NG, NJ = OP::NJ;
    const int m = face >> 1, side = face & 1;
    const T* l = s_b + (side ? BOff<NP>::LP : BOff<NP>::LM);
    const int enb = nbr_elem<D>(fe, m, side ? 1 : -1, a.nel);
    const size_t nbase = ((size_t)enb * 2 * D + (2 * m + 1 - side)) * NV * NFP + fp;
    S own[NV], nb[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        T x[NJ], y[NJ];
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
            T acc = T(0);
            if (!(AUX && j >= OP::NGLOB)) {
#pragma unroll
                for (int q = 0; q < NP; ++q) acc += l[q] * s_fld[j][fel][v][node_on_line<D, NP>(fp, m, q)];
            }
            x[j] = acc;
            const T* t = j >= OP::NGLOB ? nullptr : a.trc[j];
            y[j] = t ? t[nbase + (size_t)v * NFP] : T(0);
        }
        own[v] = OP::make(x, a);
        nb[v] = OP::make(y, a);
    }
    S go[NG], gn[NG];
    EQ::grad_vars(own, go, ep);
    EQ::grad_vars(nb, gn, ep);
#pragma unroll
    for (int k = 0; k < NG; ++k) s_jmp[((k * EPB + fel) * 2 * D + face) * NFP + fp] = (gn[k] - go[k]) * T(0.5);
}

// phase B (every node): strong gradients into s_dv
template <int D, int NP, class EQ, class OP, typename T, int EPB, int NN>
__device__ __forceinline__ void ns_strong_grad(const OpArgs<T>& a, const T* s_b, const typename OP::S* s_g,
                                               typename OP::S* s_dv, int el, int node) {
    using S = typename OP::S;
    constexpr int NG = EQ::NG;
    const int idx[3] = {node % NP, (node / NP) % NP, node / (NP * NP)};
#pragma unroll
    for (int j = 0; j < D; ++j) {
        const int ij = idx[j];
        const int stride = j == 0 ? 1 : (j == 1 ? NP : NP * NP);
        const int b0 = node - ij * stride;
        const T* Drow = s_b + BOff<NP>::DS + ij * NP;
#pragma unroll
        for (int k = 0; k < NG; ++k) {
            const S* gk = s_g + (k * EPB + el) * NN;
            S acc = gk[b0] * Drow[0];
#pragma unroll
            for (int q = 1; q < NP; ++q) acc = acc + gk[b0 + q * stride] * Drow[q];
            s_dv[((k * D + j) * EPB + el) * NN + node] = acc * a.two_h[j];
        }
    }
}

// volume gradient d at one node (global lifting)
template <int D, int NP, class EQ, class OP, typename T, int EPB, int NN, int NFP>
__device__ __forceinline__ void ns_volume_grad(const OpArgs<T>& a, const T* s_b, const typename OP::S* s_dv,
                                               const typename OP::S* s_jmp, int el, int node,
                                               typename OP::S (*d)[D]) {
    constexpr int NG = EQ::NG;
    const int idx[3] = {node % NP, (node / NP) % NP, node / (NP * NP)};
#pragma unroll
    for (int j = 0; j < D; ++j) {
        const int ij = idx[j];
        const int fpj = fp_of_node<D, NP>(node, j);
        const T lp = s_b[BOff<NP>::LHP + ij], lm = s_b[BOff<NP>::LHM + ij];
#pragma unroll
        for (int k = 0; k < NG; ++k) {
            const auto jp = s_jmp[((k * EPB + el) * 2 * D + 2 * j + 1) * NFP + fpj];
            const auto jm = s_jmp[((k * EPB + el) * 2 * D + 2 * j) * NFP + fpj];
            d[k][j] = s_dv[((k * D + j) * EPB + el) * NN + node] + (jp * lp - jm * lm) * a.two_h[j];
        }
    }
}

// the element's own BR2 gradient at a face point of its face 2M + side
template <int D, int NP, int M, class EQ, class OP, typename T, int EPB, int NN, int NFP>
__device__ __forceinline__ void ns_face_grad(const OpArgs<T>& a, const EqParams<T>& ep, const T* s_b,
                                             const typename OP::S* s_dv, const typename OP::S* s_jmp, int fel,
                                             int side, int fp, typename OP::S (*d)[D]) {
    using S = typename OP::S;
    constexpr int NG = EQ::NG, m = M;
    const T* l = s_b + (side ? BOff<NP>::LP : BOff<NP>::LM);
    const T pen = (side ? ep.eta : -ep.eta) * a.two_h[m] * s_b[side ? BOff<NP>::CP : BOff<NP>::CM];
#pragma unroll
    for (int k = 0; k < NG; ++k) {
#pragma unroll
        for (int j = 0; j < D; ++j) {
            const S* dv = s_dv + ((k * D + j) * EPB + fel) * NN;
            S acc = dv[node_on_line<D, NP>(fp, m, 0)] * l[0];
#pragma unroll
            for (int q = 1; q < NP; ++q) acc = acc + dv[node_on_line<D, NP>(fp, m, q)] * l[q];
            d[k][j] = acc;
        }
        d[k][m] = d[k][m] + s_jmp[((k * EPB + fel) * 2 * D + 2 * m + side) * NFP + fp] * pen;
    }
}

// the element's own viscous flux F^v(w, d) . e_M at a face point of its face 2M + side: w the
// trace of its fields there (jet components >= NGLOB zero), d its BR2 face gradient
template <int D, int NP, int M, class EQ, class OP, typename T, int EPB, int NN, int NFP>
__device__ __forceinline__ void ns_face_vflux(const OpArgs<T>& a, const EqParams<T>& ep, const T* s_b,
                                              const T (*s_fld)[EPB][EQ::NV][NN], const typename OP::S* s_dv,
                                              const typename OP::S* s_jmp, int fel, int side, int fp,
                                              typename OP::S* fv) {
    using S = typename OP::S;
    constexpr int NV = EQ::NV, NG = EQ::NG, NJ = OP::NJ;
    S d[NG][D];
    ns_face_grad<D, NP, M, EQ, OP, T, EPB, NN, NFP>(a, ep, s_b, s_dv, s_jmp, fel, side, fp, d);
    const T* l = s_b + (side ? BOff<NP>::LP : BOff<NP>::LM);
    S own[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        T x[NJ];
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
            T acc = T(0);
            if (j < OP::NGLOB) {
#pragma unroll
                for (int q = 0; q < NP; ++q) acc += l[q] * s_fld[j][fel][v][node_on_line<D, NP>(fp, M, q)];
            }
            x[j] = acc;
        }
        own[v] = OP::make(x, a);
    }
    EQ::viscous_flux(own, d, M, fv, ep);
}

// BR2 face-gradient kernel: for every element and face point the element's own viscous flux
// F^v(w, d) . e_m with its BR2 face gradient d (jet components j < NGLOB) into
// a.nsg[j][((e * 2D + face) * NV + v) * NFP + fp]; the operator kernel reads the neighbours'
// values from there (NV values per face point instead of the (d + 1) d of the gradient)
template <int D, int NP, class EQ, class OP, typename T>
__global__ void __launch_bounds__(256) ns_facegrad_kernel(OpArgs<T> a, EqParams<T> ep) {
    if constexpr (EQ::NS) {
        constexpr int NN = ipow(NP, D), NFP = ipow(NP, D - 1);
        constexpr int NV = EQ::NV, NJ = OP::NJ, NG = EQ::NG;
        constexpr int EPB = aux_epb<D, NP, EQ, OP, T>();
        constexpr int NT = EPB * NN;
        using S = typename OP::S;
        __shared__ T s_fld[NJ][EPB][NV][NN];
        __shared__ T s_b[basis_len<NP>()];
        __shared__ S s_g[NG * EPB * NN];
        __shared__ S s_jmp[NG * EPB * 2 * D * NFP];
        __shared__ S s_dv[NG * D * EPB * NN];
        const int tid = threadIdx.x;
        const int e0 = blockIdx.x * EPB;
        const int nloc = min(EPB, a.nE - e0);
        for (int i = tid; i < basis_len<NP>(); i += NT) s_b[i] = a.basis[i];
        for (int i = tid; i < nloc * NV * NN; i += NT) {
            const int loc = i % (NV * NN);
            const size_t g = (size_t)e0 * NV * NN + i;
#pragma unroll
            for (int j = 0; j < NJ; ++j) (&s_fld[j][0][0][0])[i] = j < OP::NGLOB ? OP::load(a, j, g, loc) : T(0);
        }
        __syncthreads();
        const int el = tid / NN, node = tid % NN;
        if (el < nloc) ns_stage_g<D, NP, EQ, OP, true, T, EPB, NN>(a, ep, s_fld, s_g, el, node);
        for (int i = tid; i < nloc * 2 * D * NFP; i += NT) {
            const int fel = i / (2 * D * NFP), r = i % (2 * D * NFP);
            ns_face_jump<D, NP, EQ, OP, true, T, EPB, NN, NFP>(a, ep, s_b, s_fld, s_jmp, fel, e0 + fel, r / NFP,
                                                                r % NFP);
        }
        __syncthreads();
        if (el < nloc) ns_strong_grad<D, NP, EQ, OP, T, EPB, NN>(a, s_b, s_g, s_dv, el, node);
        __syncthreads();
        for (int i = tid; i < nloc * 2 * D * NFP; i += NT) {
            const int fel = i / (2 * D * NFP), r = i % (2 * D * NFP);
            const int face = r / NFP, fp = r % NFP;
            S fv[NV];
            const int m = face >> 1, side = face & 1;
            if (m == 0) {
                ns_face_vflux<D, NP, 0, EQ, OP, T, EPB, NN, NFP>(a, ep, s_b, s_fld, s_dv, s_jmp, fel, side, fp, fv);
            } else if (m == 1) {
                if constexpr (D > 1)
                    ns_face_vflux<D, NP, 1, EQ, OP, T, EPB, NN, NFP>(a, ep, s_b, s_fld, s_dv, s_jmp, fel, side, fp,
                                                                      fv);
            } else {
                if constexpr (D > 2)
                    ns_face_vflux<D, NP, 2, EQ, OP, T, EPB, NN, NFP>(a, ep, s_b, s_fld, s_dv, s_jmp, fel, side, fp,
                                                                      fv);
            }
            const size_t base = ((size_t)(e0 + fel) * 2 * D + face) * NV;
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                T x[NJ];
                OP::split(fv[v], x);
#pragma unroll
                for (int c = 0; c < OP::NGLOB; ++c) a.nsg[c][(base + v) * NFP + fp] = x[c];
            }
        }
    }
}

// ----------------------------------------------------------------- operator kernel
// numerical flux at one face point of direction M (a compile-time constant, so that the state
// components indexed by M stay in registers); the side (0: the element's -e_M face, 1: its +e_M
// face) is a run-time value, so that every wave of the face phase runs one flux body whatever
// mix of sides it holds
template <int D, int NP, int M, class EQ, class OP, typename T, int EPB, int NN, int NFP>
__device__ __forceinline__ void face_point(const OpArgs<T>& a, const EqParams<T>& ep, const T* s_b,
                                           T (*s_fld)[EPB][EQ::NV][NN], T (*s_fs)[EPB][2 * D][EQ::NV][NFP],
                                           const T* s_q, const typename OP::S* s_dv, const typename OP::S* s_jmp,
                                           int fel, int fe, int fp, int side) {
    constexpr int NV = EQ::NV, NJ = OP::NJ, NC = OP::NC;
    using S = typename OP::S;
    const T* l = s_b + (side ? BOff<NP>::LP : BOff<NP>::LM);
    S own[NV], nb[NV];
    const int enb = nbr_elem<D>(fe, M, side ? 1 : -1, a.nel);
    const size_t nbase = ((size_t)enb * 2 * D + (2 * M + 1 - side)) * NV * NFP + fp;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        T x[NJ], y[NJ];
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
            T acc = T(0);
#pragma unroll
            for (int q = 0; q < NP; ++q) acc += l[q] * s_fld[j][fel][v][node_on_line<D, NP>(fp, M, q)];
            x[j] = acc;
            const T* t = j >= OP::NGLOB ? nullptr : a.trc[j];
            y[j] = t ? t[nbase + (size_t)v * NFP] : T(0);
        }
        own[v] = OP::make(x, a);
        nb[v] = OP::make(y, a);
    }
    // the element is the left state on its +e_M face and the right state on its -e_M face
    S wl[NV], wr[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        wl[v] = side ? own[v] : nb[v];
        wr[v] = side ? nb[v] : own[v];
    }
    S f[NV];
    numerical_flux<EQ>(wl, wr, M, f, ep);
    if constexpr (EQ::VISC) {
        // BR1 viscous surface flux -nu (q_L + q_R)/2 of the lifted gradient q_M
        // (s_q[j][m][el][node], NV = 1); neighbour traces of q from a.qtr
        T x[NJ], y[NJ];
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
            const T* qj = s_q + ((j * D + M) * EPB + fel) * NN;
            T acc = T(0);
#pragma unroll
            for (int q = 0; q < NP; ++q) acc += l[q] * qj[node_on_line<D, NP>(fp, M, q)];
            x[j] = acc;
            const T* t = j >= OP::NGLOB ? nullptr : a.qtr[j];
            y[j] = t ? t[((size_t)enb * 2 * D + (2 * M + 1 - side)) * NFP + fp] : T(0);
        }
        S qo = OP::make(x, a), qn = OP::make(y, a);
        f[0] = f[0] - (qo + qn) * (T(0.5) * ep.nu);
    }
    if constexpr (EQ::NS) {
        // BR2 viscous surface flux (F^v(w_own, d_own) + F^v(w_nbr, d_nbr))/2 (Eq. Riemann_visc), the
        // neighbour's flux from the face-gradient kernel
        constexpr int NG = EQ::NG;
        S dn[NG][D];
        ns_face_grad<D, NP, M, EQ, OP, T, EPB, NN, NFP>(a, ep, s_b, s_dv, s_jmp, fel, side, fp, dn);
        S fo[NV];
        EQ::viscous_flux(own, dn, M, fo, ep);
        const size_t gb = ((size_t)enb * 2 * D + (2 * M + 1 - side)) * NV;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            T y[NJ];
#pragma unroll
            for (int c = 0; c < NJ; ++c) y[c] = c < OP::NGLOB ? a.nsg[c][(gb + v) * NFP + fp] : T(0);
            f[v] = f[v] - (fo[v] + OP::make(y, a)) * T(0.5);
        }
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        T c[NC];
        OP::combo(f[v], c, a);
#pragma unroll
        for (int k = 0; k < NC; ++k) s_fs[k][fel][2 * M + side][v][fp] = c[k];
    }
}

// a0: the arguments of the first nb0 blocks; a1: those of the rest (the second system of a pair
// of stage solves, one launch for both; a single launch passes nb0 = its grid)
template <int D, int NP, class EQ, class OP, typename T>
__global__ void __launch_bounds__(256) dg_op_kernel(OpArgs<T> a0, EqParams<T> ep, OpArgs<T> a1, int nb0) {
    const bool second = (int)blockIdx.x >= nb0;
    const OpArgs<T>& a = second ? a1 : a0;
    const int bx = second ? (int)blockIdx.x - nb0 : (int)blockIdx.x;
    constexpr int NN = ipow(NP, D), NFP = ipow(NP, D - 1);
    constexpr int NV = EQ::NV, NJ = OP::NJ, NC = OP::NC;
    constexpr int EPB = kernel_epb<D, NP, EQ, OP, T>();
    constexpr int NT = EPB * NN;
    using S = typename OP::S;

    __shared__ T s_fld[NJ][EPB][NV][NN];
    constexpr int NG = eq_ng<EQ>();                      // BR2 (Navier-Stokes) lifting in LDS
    __shared__ S s_g[NG > 0 ? NG * EPB * NN : 1];
    __shared__ S s_jmp[NG > 0 ? NG * EPB * 2 * D * NFP : 1];
    __shared__ S s_dv[NG > 0 ? NG * D * EPB * NN : 1];
    __shared__ T s_flx[NC][EPB][NV][NN];                 // flux combinations of one direction
    __shared__ T s_fs[NC][EPB][2 * D][NV][NFP];
    __shared__ T s_b[basis_len<NP>()];
    constexpr int NQ = EQ::VISC ? NJ : 0;                 // BR1: lifted gradients of the jet fields
    __shared__ T s_q[NQ > 0 ? NQ * D * EPB * NN : 1];     // [j][m][el][node]
    __shared__ T s_us[NQ > 0 ? NQ * EPB * 2 * D * NFP : 1];   // u* = (u_own + u_nbr)/2 at face points

    const int tid = threadIdx.x;
    const int e0 = a.e_begin + bx * EPB;
    const int nloc = min(EPB, a.e_end - e0);

    // 1) stage the 1-D operators and the jet fields of EPB consecutive elements
    for (int i = tid; i < basis_len<NP>(); i += NT) s_b[i] = a.basis[i];
    for (int i = tid; i < nloc * NV * NN; i += NT) {
        int loc = i % (NV * NN);
        size_t g = (size_t)e0 * NV * NN + i;
#pragma unroll
        for (int j = 0; j < NJ; ++j) (&s_fld[j][0][0][0])[i] = OP::load(a, j, g, loc);
    }
    __syncthreads();

    const int el = tid / NN, node = tid % NN;
    const bool valid = el < nloc;

    if constexpr (EQ::NS) {
        // 1b) BR2: g at the nodes, jumps at the face points, then the strong gradients
        if (valid) ns_stage_g<D, NP, EQ, OP, false, T, EPB, NN>(a, ep, s_fld, s_g, el, node);
        for (int i = tid; i < nloc * 2 * D * NFP; i += NT) {
            const int fel = i / (2 * D * NFP), r = i % (2 * D * NFP);
            ns_face_jump<D, NP, EQ, OP, false, T, EPB, NN, NFP>(a, ep, s_b, s_fld, s_jmp, fel, e0 + fel, r / NFP,
                                                                 r % NFP);
        }
        __syncthreads();
        if (valid) ns_strong_grad<D, NP, EQ, OP, T, EPB, NN>(a, s_b, s_g, s_dv, el, node);
        __syncthreads();
    }

    if constexpr (EQ::VISC) {
        // 1b) BR1 lifting q_m = (2/h_m)[Dhat u + lhat(+1) u*_+ - lhat(-1) u*_-], u* central
        for (int i = tid; i < nloc * 2 * D * NFP; i += NT) {
            const int fel = i / (2 * D * NFP), r = i % (2 * D * NFP);
            const int face = r / NFP, fp = r % NFP;
            const int m = face >> 1, side = face & 1;
            const T* l = s_b + (side ? BOff<NP>::LP : BOff<NP>::LM);
            const int enb = nbr_elem<D>(e0 + fel, m, side ? 1 : -1, a.nel);
            const size_t nb = ((size_t)enb * 2 * D + (2 * m + 1 - side)) * NFP + fp;
#pragma unroll
            for (int j = 0; j < NJ; ++j) {
                T own = T(0);
                for (int q = 0; q < NP; ++q) own += l[q] * s_fld[j][fel][0][node_on_line<D, NP>(fp, m, q)];
                const T* t = j >= OP::NGLOB ? nullptr : a.trc[j];
                const T nbv = t ? t[nb] : T(0);
                s_us[((j * EPB + fel) * 2 * D + face) * NFP + fp] = T(0.5) * (own + nbv);
            }
        }
        __syncthreads();
        if (valid) {
            const int id3[3] = {node % NP, (node / NP) % NP, node / (NP * NP)};
#pragma unroll
            for (int j = 0; j < NJ; ++j)
#pragma unroll
                for (int m = 0; m < D; ++m) {
                    const int im = id3[m];
                    const int stride = m == 0 ? 1 : (m == 1 ? NP : NP * NP);
                    const int b0 = node - im * stride;
                    const T* Drow = s_b + BOff<NP>::D + im * NP;
                    T sv = T(0);
                    for (int q = 0; q < NP; ++q) sv += Drow[q] * s_fld[j][el][0][b0 + q * stride];
                    const int fpm = fp_of_node<D, NP>(node, m);
                    const T* us = s_us + ((j * EPB + el) * 2 * D + 2 * m) * NFP;
                    sv += s_b[BOff<NP>::LHP + im] * us[NFP + fpm] - s_b[BOff<NP>::LHM + im] * us[fpm];
                    s_q[((j * D + m) * EPB + el) * NN + node] = a.two_h[m] * sv;
                }
        }
        __syncthreads();
    }

    // 2) numerical fluxes at the face points (own trace from LDS, neighbour trace from HBM); items
    //    ordered (direction, element, side, face point), so that a wave holds one direction (two
    //    where it straddles a direction boundary) and evaluates one flux body per direction
    constexpr int PER_M = 2 * NFP;
    const int per_dir = nloc * PER_M;
    for (int i = tid; i < D * per_dir; i += NT) {
        const int m = i / per_dir, r = i % per_dir;
        const int fel = r / PER_M, r2 = r % PER_M;
        const int side = r2 / NFP, fp = r2 % NFP;
        const int fe = e0 + fel;
        if (m == 0) {
            face_point<D, NP, 0, EQ, OP, T, EPB, NN, NFP>(a, ep, s_b, s_fld, s_fs, s_q, s_dv, s_jmp, fel, fe, fp,
                                                               side);
        } else if (m == 1) {
            if constexpr (D > 1)
                face_point<D, NP, 1, EQ, OP, T, EPB, NN, NFP>(a, ep, s_b, s_fld, s_fs, s_q, s_dv, s_jmp, fel, fe, fp,
                                                               side);
        } else {
            if constexpr (D > 2)
                face_point<D, NP, 2, EQ, OP, T, EPB, NN, NFP>(a, ep, s_b, s_fld, s_fs, s_q, s_dv, s_jmp, fel, fe, fp,
                                                               side);
        }
    }

    // 3) jet-valued volume fluxes at this node, kept in registers
    S F[D][NV];
    if (valid) {
        S wn[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            T x[NJ];
#pragma unroll
            for (int j = 0; j < NJ; ++j) x[j] = s_fld[j][el][v][node];
            wn[v] = OP::make(x, a);
        }
        EQ::flux_all(wn, F, ep);
        if constexpr (EQ::NS) {
            // minus the viscous flux of the volume gradient (global lifting)
            S d[eq_ng<EQ>()][D];
            ns_volume_grad<D, NP, EQ, OP, T, EPB, NN, NFP>(a, s_b, s_dv, s_jmp, el, node, d);
#pragma unroll
            for (int m = 0; m < D; ++m) {
                S Fv[NV];
                EQ::viscous_flux(wn, d, m, Fv, ep);
#pragma unroll
                for (int v = 0; v < NV; ++v) F[m][v] = F[m][v] - Fv[v];
            }
        }
        if constexpr (EQ::VISC) {
#pragma unroll
            for (int m = 0; m < D; ++m) {
                T x[NJ];
#pragma unroll
                for (int j = 0; j < NJ; ++j) x[j] = s_q[((j * D + m) * EPB + el) * NN + node];
                F[m][0] = F[m][0] - OP::make(x, a) * ep.nu;
            }
        }
    }

    // 4) per direction m: the flux combinations of F_m to LDS, then the D-hat sweep along m and the
    //    surface lifting of faces 2m, 2m+1, summed over m in increasing order
    const int idx[3] = {node % NP, (node / NP) % NP, node / (NP * NP)};
    T acc[NV][NC];
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
        for (int k = 0; k < NC; ++k) acc[v][k] = T(0);
#pragma unroll
    for (int m = 0; m < D; ++m) {
        if (m > 0) __syncthreads();   // the previous direction's sweep has read s_flx
        if (valid) {
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                T c[NC];
                OP::combo(F[m][v], c, a);
#pragma unroll
                for (int k = 0; k < NC; ++k) s_flx[k][el][v][node] = c[k];
            }
        }
        __syncthreads();   // s_flx of direction m and (first pass) the face fluxes are in LDS
        if (valid) {
            const int im = idx[m];
            const int stride = m == 0 ? 1 : (m == 1 ? NP : NP * NP);
            const int b0 = node - im * stride;
            const T* Drow = s_b + BOff<NP>::D + im * NP;
            const int fp = fp_of_node<D, NP>(node, m);
#pragma unroll
            for (int v = 0; v < NV; ++v)
#pragma unroll
                for (int k = 0; k < NC; ++k) {
                    T sm = T(0);
#pragma unroll
                    for (int q = 0; q < NP; ++q) sm += Drow[q] * s_flx[k][el][v][b0 + q * stride];
                    sm += s_b[BOff<NP>::LHP + im] * s_fs[k][el][2 * m + 1][v][fp] -
                          s_b[BOff<NP>::LHM + im] * s_fs[k][el][2 * m][v][fp];
                    acc[v][k] += a.two_h[m] * sm;
                }
        }
    }
    if (!valid) return;
    const int e = e0 + el;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        T gv[NC];
#pragma unroll
        for (int k = 0; k < NC; ++k) gv[k] = -acc[v][k];
        const int loc = v * NN + node;
        OP::output(a, (size_t)e * NV * NN + loc, e, loc, gv);
    }
}
