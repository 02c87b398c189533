// BJ_ext preconditioner kernels (Sec. 3.2.3).
//
// Build: from the element-local Jacobians K_i (stored column-major, KT[e][c][r]
// = K_i[r][c], produced column by column by the KCOL operator kernel), form
// S_i = I - a1dt K_i + bcoef K_i^2 in registers and invert it by Gauss-Jordan
// elimination with partial pivoting; store S_i^-1 column-major (SinvT[e][c][r]).
// One workgroup of TG x TG threads per element; thread (tr, tc) owns rows
// tr + TG a and columns tc + TG b (a, b < R), so blocks up to R*TG fit.
//
// Apply: the local products K vs and K (vw - a1dt vs) come from the PCPRE
// operator kernel (a = vw - bcoef K vs, c = vs + K (vw - a1dt vs)); since S_i
// is a polynomial in K_i, S^-1 commutes with K and
//   P^-1 (vw, vs) = (D vw + E vs, F vw + G vs) = (S^-1 a, S^-1 c).
#include <hip/hip_runtime.h>
#include <cstdint>

template <int TGR, int TGC, int RR, int RC, typename T, typename TO>
__global__ void __launch_bounds__(TGR* TGC) bj_invert_kernel(const T* __restrict__ KT, TO* __restrict__ SinvT,
                                                            int NE, T a1dt, T bc, int* __restrict__ status) {
    // thread (tr, tc), tid = tr + TGR tc, owns rows tr + TGR a (a < RR) and
    // columns tc + TGC b (b < RC); a column group (fixed tc) is TGR
    // consecutive lanes of one wave.  Register indices are compile-time
    // constants throughout (runtime indices would move acc[][] to scratch).
    constexpr int NT = TGR * TGC;
    constexpr int KC = 8;
    constexpr int NRMAX = TGR * RR;
    constexpr int NCMAX = TGC * RC;
    constexpr int NMAX = NRMAX > NCMAX ? NRMAX : NCMAX;
    __shared__ T sA[KC][NMAX];   // K[r][kk+t]
    __shared__ T sB[KC][NMAX];   // K[kk+t][c]
    __shared__ T s_row[NMAX];    // pivot row p
    __shared__ T s_col[NMAX];    // column k
    __shared__ int s_prow[NMAX]; // pivot row of step k
    __shared__ int s_pinv[NMAX]; // step at which row r was pivot
    __shared__ int s_p;

    const int tid = threadIdx.x;
    const int tr = tid % TGR, tc = tid / TGR;
    const size_t e = blockIdx.x;
    const T* K = KT + e * (size_t)NE * NE;

    T acc[RR][RC];
#pragma unroll
    for (int a = 0; a < RR; ++a)
#pragma unroll
        for (int b = 0; b < RC; ++b) acc[a][b] = T(0);

    // ---- K^2 for the owned entries, K staged through LDS in slabs of KC
    for (int kk = 0; kk < NE; kk += KC) {
        for (int i = tid; i < KC * NE; i += NT) {
            int t = i / NE, x = i % NE;
            int k = kk + t;
            sA[t][x] = k < NE ? K[(size_t)k * NE + x] : T(0);   // K[x][k] = KT[k][x]
        }
        for (int i = tid; i < KC * NE; i += NT) {
            int x = i / KC, t = i % KC;                      // consecutive threads: consecutive k
            int k = kk + t;
            sB[t][x] = k < NE ? K[(size_t)x * NE + k] : T(0);   // K[k][x] = KT[x][k]
        }
        __syncthreads();
#pragma unroll
        for (int t = 0; t < KC; ++t) {
            T ra[RR], cb[RC];
#pragma unroll
            for (int a = 0; a < RR; ++a) ra[a] = sA[t][(tr + TGR * a) < NE ? tr + TGR * a : 0];
#pragma unroll
            for (int b = 0; b < RC; ++b) cb[b] = sB[t][(tc + TGC * b) < NE ? tc + TGC * b : 0];
#pragma unroll
            for (int a = 0; a < RR; ++a)
#pragma unroll
                for (int b = 0; b < RC; ++b) acc[a][b] += ra[a] * cb[b];
        }
        __syncthreads();
    }
    // ---- S = I - a1dt K + bc K^2 (padding rows/columns: identity, never used)
    unsigned used = 0u;   // bit a: owned row a has been a pivot row
#pragma unroll
    for (int a = 0; a < RR; ++a)
#pragma unroll
        for (int b = 0; b < RC; ++b) {
            int r = tr + TGR * a, c = tc + TGC * b;
            T v = (r == c) ? T(1) : T(0);
            if (r < NE && c < NE) v += -a1dt * K[(size_t)c * NE + r] + bc * acc[a][b];
            acc[a][b] = v;
        }

    // ---- Gauss-Jordan exchange steps without row swaps: step k pivots on
    // (p_k, k) with p_k the largest unused entry of column k; afterwards
    // S^-1[k][p_j] = T[p_k][j].
    for (int k = 0; k < NE; ++k) {
        const int ck = k % TGC, bk = k / TGC;
        if (tc == ck) {
            T best = T(-1);
            int bi = NE;
#pragma unroll
            for (int a = 0; a < RR; ++a) {
                const int r = tr + TGR * a;
                T v = T(0);
#pragma unroll
                for (int b = 0; b < RC; ++b) v = (b == bk) ? acc[a][b] : v;
                v = v >= T(0) ? v : -v;
                const bool take = r < NE && !((used >> a) & 1u) && v > best;
                best = take ? v : best;
                bi = take ? r : bi;
            }
#pragma unroll
            for (int off = 1; off < TGR; off <<= 1) {
                T ob = __shfl_xor(best, off, TGR);
                int oi = __shfl_xor(bi, off, TGR);
                if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
            }
            if (tr == 0) s_p = bi;
        }
        __syncthreads();
        const int p = s_p;
        if (p >= NE) {                     // no finite pivot left: flag, stop
            if (tid == 0) atomicOr(status, 1);
            return;
        }
        if (tid == 0) {
            s_prow[k] = p;
            s_pinv[p] = k;
        }
        const int ap = p / TGR;
        if (tr == p % TGR) {               // owners of row p publish it
            used |= 1u << ap;
#pragma unroll
            for (int b = 0; b < RC; ++b) {
                const int c = tc + TGC * b;
                T v = T(0);
#pragma unroll
                for (int a = 0; a < RR; ++a) v = (a == ap) ? acc[a][b] : v;
                if (c < NE) s_row[c] = v;
            }
        }
        if (tc == ck) {                    // owners of column k publish it
#pragma unroll
            for (int a = 0; a < RR; ++a) {
                const int r = tr + TGR * a;
                T v = T(0);
#pragma unroll
                for (int b = 0; b < RC; ++b) v = (b == bk) ? acc[a][b] : v;
                if (r < NE) s_col[r] = v;
            }
        }
        __syncthreads();
        const T piv = s_col[p];
        const T ipiv = T(1) / piv;
        if (!(piv == piv) || piv == T(0)) {
            if (tid == 0) atomicOr(status, 1);
        }
        T pr[RC], f[RR];
#pragma unroll
        for (int b = 0; b < RC; ++b) {
            const int c = tc + TGC * b;
            pr[b] = c < NE ? s_row[c] * ipiv : T(0);
        }
#pragma unroll
        for (int a = 0; a < RR; ++a) {
            const int r = tr + TGR * a;
            f[a] = r < NE ? s_col[r] : T(0);
        }
        // branch-free update (selects only): pivot row / pivot column / the rest
#pragma unroll
        for (int a = 0; a < RR; ++a) {
            const bool isp = (tr + TGR * a == p);
            const T fcol = -f[a] * ipiv;
            const T pk = isp ? ipiv : fcol;
#pragma unroll
            for (int b = 0; b < RC; ++b) {
                const bool isk = (tc + TGC * b == k);
                const T upd = acc[a][b] - f[a] * pr[b];
                const T v = isp ? pr[b] : upd;
                acc[a][b] = isk ? pk : v;
            }
        }
        __syncthreads();
    }
    // ---- S^-1[pinv[r]][prow[c]] = T[r][c], stored column-major (SinvT[col][row])
    TO* out = SinvT + e * (size_t)NE * NE;
#pragma unroll
    for (int b = 0; b < RC; ++b) {
        const int c = tc + TGC * b;
        if (c >= NE) continue;
        const int col = s_prow[c];
#pragma unroll
        for (int a = 0; a < RR; ++a) {
            const int r = tr + TGR * a;
            if (r < NE) out[(size_t)col * NE + s_pinv[r]] = (TO)acc[a][b];
        }
    }
}

// y = S^-1 x for the two right-hand sides (w block, sigma block); one thread per row.
template <typename TM, typename T>
__global__ void __launch_bounds__(256) bj_apply_kernel(const TM* __restrict__ SinvT, const T* __restrict__ xa,
                                                      const T* __restrict__ xc, T* __restrict__ yw,
                                                      T* __restrict__ ys, int NE, int nE) {
    extern __shared__ unsigned char smem_raw[];
    T* sx = reinterpret_cast<T*>(smem_raw);
    const int epb = blockDim.x / NE;
    const int el = threadIdx.x / NE, r = threadIdx.x % NE;
    const int e0 = blockIdx.x * epb;
    for (int i = threadIdx.x; i < epb * NE; i += blockDim.x) {
        int le = i / NE;
        size_t g = (size_t)(e0 + le) * NE + (i % NE);
        bool ok = e0 + le < nE;
        sx[2 * i] = ok ? xa[g] : T(0);
        sx[2 * i + 1] = ok ? xc[g] : T(0);
    }
    __syncthreads();
    const int e = e0 + el;
    if (el >= epb || e >= nE) return;
    const TM* M = SinvT + (size_t)e * NE * NE + r;
    const T* x = sx + 2 * el * NE;
    T s0 = T(0), s1 = T(0);
    int c = 0;
    for (; c + 4 <= NE; c += 4) {
        T m0 = (T)M[(size_t)(c + 0) * NE], m1 = (T)M[(size_t)(c + 1) * NE];
        T m2 = (T)M[(size_t)(c + 2) * NE], m3 = (T)M[(size_t)(c + 3) * NE];
        s0 += m0 * x[2 * c + 0] + m1 * x[2 * c + 2] + m2 * x[2 * c + 4] + m3 * x[2 * c + 6];
        s1 += m0 * x[2 * c + 1] + m1 * x[2 * c + 3] + m2 * x[2 * c + 5] + m3 * x[2 * c + 7];
    }
    for (; c < NE; ++c) {
        T m = (T)M[(size_t)c * NE];
        s0 += m * x[2 * c];
        s1 += m * x[2 * c + 1];
    }
    yw[(size_t)e * NE + r] = s0;
    ys[(size_t)e * NE + r] = s1;
}

template <int TGR, int TGC, int RR, int RC, typename TO>
static hipError_t launch_inv(const double* KT, TO* SinvT, int NE, int nE, double a1dt, double bc, int* status,
                             hipStream_t st) {
    hipLaunchKernelGGL((bj_invert_kernel<TGR, TGC, RR, RC, double, TO>), dim3(nE), dim3(TGR * TGC), 0, st, KT,
                       SinvT, NE, a1dt, bc, status);
    return hipGetLastError();
}

hipError_t bj_invert(const double* KT, void* SinvT, int f32, int NE, int nE, double a1dt, double bc, int* status,
                     hipStream_t st) {
    if (nE == 0) return hipSuccess;
#define HBPC_INV(TGR, TGC, RR, RC)                                                                         \
    return f32 ? launch_inv<TGR, TGC, RR, RC, float>(KT, (float*)SinvT, NE, nE, a1dt, bc, status, st)    \
               : launch_inv<TGR, TGC, RR, RC, double>(KT, (double*)SinvT, NE, nE, a1dt, bc, status, st);
    if (NE <= 16) { HBPC_INV(4, 4, 4, 4) }
    if (NE <= 32) { HBPC_INV(8, 8, 4, 4) }
    if (NE <= 64) { HBPC_INV(16, 16, 4, 4) }
    if (NE <= 144) { HBPC_INV(16, 32, 9, 5) }
#undef HBPC_INV
    return hipErrorInvalidValue;
}

hipError_t bj_apply(const void* SinvT, int m_f32, const void* xa, const void* xc, void* yw, void* ys, int v_f32,
                    int NE, int nE, hipStream_t st) {
    if (nE == 0) return hipSuccess;
    int epb = NE >= 256 ? 1 : 256 / NE;
    int threads = epb * NE;
    if (threads > 1024) return hipErrorInvalidValue;
    int grid = (nE + epb - 1) / epb;
    size_t sh = (size_t)2 * epb * NE * (v_f32 ? sizeof(float) : sizeof(double));
    if (v_f32) {
        if (m_f32)
            hipLaunchKernelGGL((bj_apply_kernel<float, float>), dim3(grid), dim3(threads), sh, st,
                               (const float*)SinvT, (const float*)xa, (const float*)xc, (float*)yw, (float*)ys, NE, nE);
        else
            hipLaunchKernelGGL((bj_apply_kernel<double, float>), dim3(grid), dim3(threads), sh, st,
                               (const double*)SinvT, (const float*)xa, (const float*)xc, (float*)yw, (float*)ys, NE,
                               nE);
    } else {
        if (m_f32)
            hipLaunchKernelGGL((bj_apply_kernel<float, double>), dim3(grid), dim3(threads), sh, st,
                               (const float*)SinvT, (const double*)xa, (const double*)xc, (double*)yw, (double*)ys,
                               NE, nE);
        else
            hipLaunchKernelGGL((bj_apply_kernel<double, double>), dim3(grid), dim3(threads), sh, st,
                               (const double*)SinvT, (const double*)xa, (const double*)xc, (double*)yw, (double*)ys,
                               NE, nE);
    }
    return hipGetLastError();
}
