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

template <int TG, int R, typename T, typename TO>
__global__ void __launch_bounds__(TG* TG) bj_invert_kernel(const T* __restrict__ KT, TO* __restrict__ SinvT, int NE,
                                                          T a1dt, T bc, int* __restrict__ status) {
    constexpr int NT = TG * TG;
    constexpr int KC = 8;
    constexpr int NMAX = TG * R;
    __shared__ T sA[KC][NMAX];   // K[r][kk+t]
    __shared__ T sB[KC][NMAX];   // K[kk+t][c]
    __shared__ T s_row[NMAX];
    __shared__ T s_rowk[NMAX];
    __shared__ T s_col[NMAX];
    __shared__ int s_piv[NMAX];
    __shared__ int s_perm[NMAX];
    __shared__ int s_p;

    const int tid = threadIdx.x;
    const int tr = tid % TG, tc = tid / TG;
    const size_t e = blockIdx.x;
    const T* K = KT + e * (size_t)NE * NE;

    T acc[R][R];
#pragma unroll
    for (int a = 0; a < R; ++a)
#pragma unroll
        for (int b = 0; b < R; ++b) acc[a][b] = T(0);

    // ---- K^2 (rows owned x cols owned), staged through LDS in slabs of KC
    for (int kk = 0; kk < NE; kk += KC) {
        for (int i = tid; i < KC * NE; i += NT) {
            int t = i / NE, x = i % NE;
            int k = kk + t;
            sA[t][x] = k < NE ? K[(size_t)k * NE + x] : T(0);   // K[x][k] = KT[k][x]
            sB[t][x] = k < NE ? K[(size_t)x * NE + k] : T(0);   // K[k][x] = KT[x][k]
        }
        __syncthreads();
#pragma unroll
        for (int t = 0; t < KC; ++t) {
            T ra[R], cb[R];
#pragma unroll
            for (int a = 0; a < R; ++a) ra[a] = (tr + TG * a) < NE ? sA[t][tr + TG * a] : T(0);
#pragma unroll
            for (int b = 0; b < R; ++b) cb[b] = (tc + TG * b) < NE ? sB[t][tc + TG * b] : T(0);
#pragma unroll
            for (int a = 0; a < R; ++a)
#pragma unroll
                for (int b = 0; b < R; ++b) acc[a][b] += ra[a] * cb[b];
        }
        __syncthreads();
    }
    // ---- S = I - a1dt K + bc K^2 (padding rows/cols: identity)
#pragma unroll
    for (int a = 0; a < R; ++a)
#pragma unroll
        for (int b = 0; b < R; ++b) {
            int r = tr + TG * a, c = tc + TG * b;
            T v = (r == c) ? T(1) : T(0);
            if (r < NE && c < NE) v += -a1dt * K[(size_t)c * NE + r] + bc * acc[a][b];
            acc[a][b] = v;
        }

    // ---- Gauss-Jordan with partial pivoting, in place.  Every register index is
    // a compile-time constant (runtime indices would move acc[][] to scratch).
    for (int k = 0; k < NE; ++k) {
        const int ck = k % TG, bk = k / TG;
        if (tc == ck) {
            T best = T(-1);
            int bi = NE;
#pragma unroll
            for (int a = 0; a < R; ++a) {
                const int r = tr + TG * a;
                T v = T(0);
#pragma unroll
                for (int b = 0; b < R; ++b) v = (b == bk) ? acc[a][b] : v;
                v = v >= T(0) ? v : -v;
                if (r >= k && r < NE && v > best) { best = v; bi = r; }
            }
            // reduce over the TG threads of this column group (consecutive lanes)
#pragma unroll
            for (int off = 1; off < TG; off <<= 1) {
                T ob = __shfl_xor(best, off, TG);
                int oi = __shfl_xor(bi, off, TG);
                if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
            }
            if (tr == 0) s_p = bi < NE ? bi : k;   // all-NaN column: keep k, flagged below
        }
        __syncthreads();
        const int p = s_p;
        if (tid == 0) s_piv[k] = p;
        // publish row p, row k and column k
#pragma unroll
        for (int a = 0; a < R; ++a) {
            const int r = tr + TG * a;
#pragma unroll
            for (int b = 0; b < R; ++b) {
                const int c = tc + TG * b;
                if (c < NE) {
                    if (r == p) s_row[c] = acc[a][b];
                    if (r == k) s_rowk[c] = acc[a][b];
                }
                if (c == k && r < NE) s_col[r] = acc[a][b];
            }
        }
        __syncthreads();
        const T piv = s_col[p];
        const T ipiv = T(1) / piv;
        T pr[R], rk[R], f[R];
#pragma unroll
        for (int b = 0; b < R; ++b) {
            const int c = tc + TG * b;
            const bool in = c < NE;
            pr[b] = (c == k) ? ipiv : (in ? s_row[c] * ipiv : T(0));   // new pivot row / pivot
            rk[b] = in ? s_rowk[c] : T(0);                              // old row k (moves to row p)
        }
#pragma unroll
        for (int a = 0; a < R; ++a) {
            const int r = tr + TG * a;
            f[a] = (r < NE) ? (r == p ? s_col[k] : s_col[r]) : T(0);  // multiplier A'[r][k]
        }
#pragma unroll
        for (int a = 0; a < R; ++a) {
            const int r = tr + TG * a;
#pragma unroll
            for (int b = 0; b < R; ++b) {
                const int c = tc + TG * b;
                T cur = (r == p) ? rk[b] : acc[a][b];
                cur = (c == k) ? T(0) : cur;
                T upd = cur - f[a] * pr[b];
                acc[a][b] = (r == k) ? pr[b] : upd;
            }
        }
        if (!(piv == piv) || piv == T(0)) {
            if (tid == 0) atomicOr(status, 1);
        }
        __syncthreads();
    }
    // ---- undo the column permutation: S^-1 = A P, swaps applied in reverse order
    if (tid == 0) {
        for (int j = 0; j < NE; ++j) s_perm[j] = j;
        for (int k = NE - 1; k >= 0; --k) {
            int p = s_piv[k];
            int t = s_perm[k];
            s_perm[k] = s_perm[p];
            s_perm[p] = t;
        }
        // invert the permutation in place into s_piv
        for (int j = 0; j < NE; ++j) s_piv[s_perm[j]] = j;
    }
    __syncthreads();
    TO* out = SinvT + e * (size_t)NE * NE;
#pragma unroll
    for (int b = 0; b < R; ++b) {
        int c = tc + TG * b;
        if (c >= NE) continue;
        int j = s_piv[c];
#pragma unroll
        for (int a = 0; a < R; ++a) {
            int r = tr + TG * a;
            if (r < NE) out[(size_t)j * NE + r] = (TO)acc[a][b];
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

template <int TG, int R, typename TO>
static hipError_t launch_inv(const double* KT, TO* SinvT, int NE, int nE, double a1dt, double bc, int* status,
                             hipStream_t st) {
    hipLaunchKernelGGL((bj_invert_kernel<TG, R, double, TO>), dim3(nE), dim3(TG * TG), 0, st, KT, SinvT, NE,
                       a1dt, bc, status);
    return hipGetLastError();
}

hipError_t bj_invert(const double* KT, void* SinvT, int f32, int NE, int nE, double a1dt, double bc, int* status,
                     hipStream_t st) {
    if (nE == 0) return hipSuccess;
    if (NE <= 16) {
        return f32 ? launch_inv<4, 4, float>(KT, (float*)SinvT, NE, nE, a1dt, bc, status, st)
                   : launch_inv<4, 4, double>(KT, (double*)SinvT, NE, nE, a1dt, bc, status, st);
    }
    if (NE <= 32) {
        return f32 ? launch_inv<8, 4, float>(KT, (float*)SinvT, NE, nE, a1dt, bc, status, st)
                   : launch_inv<8, 4, double>(KT, (double*)SinvT, NE, nE, a1dt, bc, status, st);
    }
    if (NE <= 64) {
        return f32 ? launch_inv<16, 4, float>(KT, (float*)SinvT, NE, nE, a1dt, bc, status, st)
                   : launch_inv<16, 4, double>(KT, (double*)SinvT, NE, nE, a1dt, bc, status, st);
    }
    if (NE <= 144) {
        return f32 ? launch_inv<16, 9, float>(KT, (float*)SinvT, NE, nE, a1dt, bc, status, st)
                   : launch_inv<16, 9, double>(KT, (double*)SinvT, NE, nE, a1dt, bc, status, st);
    }
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
