// BJ_ext preconditioner build (Sec. 3.2.3).
//
// From the element-local Jacobians K_i (stored column-major, KT[e][c][r]
// = K_i[r][c], FP64, produced column by column by the KCOL operator kernel), form
// S_i = I - a1dt K_i + bcoef K_i^2 (BJ_ext), or with the element-local Hessian
// block H_i (HT, same layout, optional) S_i = I - a1dt K_i + bcoef (K_i^2 + H_i)
// (BJ^H_ext), and invert it by Gauss-Jordan
// elimination with partial pivoting, in the precision S_i^-1 is stored in;
// store S_i^-1 column-major (SinvT[e][c][r]).
// Blocks up to 144 unknowns: one workgroup of TG x TG threads per element, the
// matrix in registers; thread (tr, tc) owns rows tr + TG a and columns tc + TG b.
// Larger blocks (up to 1024): the blocked kernel below, matrix in the output.

#include <hip/hip_runtime.h>
#include <cstdint>
#include <type_traits>

template <int TGR, int TGC, int RR, int RC, typename T, typename TO>
__global__ void __launch_bounds__(TGR* TGC) bj_invert_kernel(const double* __restrict__ KT,
                                                            const double* __restrict__ HT, TO* __restrict__ SinvT,
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
    const double* K = KT + e * (size_t)NE * NE;
    const double* Hm = HT ? HT + e * (size_t)NE * NE : nullptr;

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
            sA[t][x] = k < NE ? (T)K[(size_t)k * NE + x] : T(0);   // K[x][k] = KT[k][x]
        }
        for (int i = tid; i < KC * NE; i += NT) {
            int x = i / KC, t = i % KC;                      // consecutive threads: consecutive k
            int k = kk + t;
            sB[t][x] = k < NE ? (T)K[(size_t)x * NE + k] : T(0);   // K[k][x] = KT[x][k]
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
    // ---- S = I - a1dt K + bc (K^2 + H) (padding rows/columns: identity, never used)
    unsigned used = 0u;   // bit a: owned row a has been a pivot row
#pragma unroll
    for (int a = 0; a < RR; ++a)
#pragma unroll
        for (int b = 0; b < RC; ++b) {
            int r = tr + TGR * a, c = tc + TGC * b;
            T v = (r == c) ? T(1) : T(0);
            if (r < NE && c < NE) {
                T h = Hm ? (T)Hm[(size_t)c * NE + r] : T(0);
                v += -a1dt * (T)K[(size_t)c * NE + r] + bc * (acc[a][b] + h);
            }
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
            if (r < NE) {
                if constexpr (sizeof(TO) == 2) {   // half storage: an entry beyond its range is flagged
                    if (!(acc[a][b] <= T(65504) && acc[a][b] >= T(-65504))) atomicOr(status, 1);
                }
                out[(size_t)col * NE + s_pinv[r]] = (TO)acc[a][b];
            }
        }
    }
}

// ---- element blocks too large for registers (the 3-D Euler N = 3 block has 320 unknowns):
// blocked Gauss-Jordan with the working matrix A (column-major, A[c * NE + r]) kept in the
// element's output block.  Panels of PB columns are eliminated in registers (lane pr of wave pc
// holds rows pr + 64 a and panel columns pc + 4 b, so one wave owns whole columns and finds a
// pivot alone) with the same pivot rule as the register kernel (largest not-yet-pivot entry of
// the column, smallest row on ties), then copied to LDS as the update's left factor.
// A run of exchange steps on distinct rows P and columns Q composes into one block exchange:
// with M = the panel columns after elimination and U = A[P][c] before it, every column c
// outside the panel becomes A[r][c] <- [r not in P] A[r][c] + sum_j M[r][j] U[j][c].
// The K^2 product and the update run in 64 x 64 output tiles; thread (tr, tc) owns rows
// r0 + 4 tr + i (i < 4) and columns c0 + tc + 16 b (b < 4).  At the end the element's K slot
// (no longer needed) holds a copy of A for the row/column permutation into S^-1.
constexpr int BIG_THREADS = 256;
constexpr int BIG_TILE = 64;
constexpr int BIG_KC = 16;

template <typename T> struct BigLds {
    int nep, pb;                 // padded row pitch of a panel column, panel width
    size_t off_u, off_col, off_row, off_ired, off_prow, off_pinv, bytes;
};

template <typename T> __host__ __device__ inline BigLds<T> big_lds(int NE, int pb) {
    BigLds<T> L;
    L.nep = (NE + 3) / 4 * 4;
    L.pb = pb;
    size_t p = (size_t)pb * L.nep;                               // panel, or the two K^2 staging tiles
    const size_t stage = (size_t)BIG_KC * BIG_TILE + (size_t)BIG_KC * (BIG_TILE + 1);
    if (p < stage) p = stage;
    size_t off = p * sizeof(T);
    L.off_u = off;    off += (size_t)pb * BIG_TILE * sizeof(T);
    L.off_col = off;  off += (size_t)L.nep * sizeof(T);
    L.off_row = off;  off += (size_t)pb * sizeof(T);
    L.off_ired = off; off += 8 * sizeof(int);
    L.off_prow = off; off += (size_t)NE * sizeof(int);
    L.off_pinv = off; off += (size_t)NE * sizeof(int);
    L.bytes = off;
    return L;
}

// argmax over the 64 lanes of a wave: largest value, smallest index on ties
template <typename T> __device__ __forceinline__ void wave_argmax(T& best, int& bi) {
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const T ob = __shfl_xor(best, off, 64);
        const int oi = __shfl_xor(bi, off, 64);
        if (ob > best || (ob == best && oi < bi)) {
            best = ob;
            bi = oi;
        }
    }
}

// rows rb .. rb+3 of one column (zeros outside the block); v4: NE % 4 == 0, so the four values
// are in range together and 16-byte aligned
template <typename T>
__device__ __forceinline__ void load_rows4(const T* col, int rb, int NE, bool colok, bool v4, T* out) {
    if (!colok || rb >= NE) {
#pragma unroll
        for (int i = 0; i < 4; ++i) out[i] = T(0);
    } else if (v4) {
        if constexpr (sizeof(T) == 4) {
            const float4 v = *reinterpret_cast<const float4*>(col + rb);
            out[0] = v.x; out[1] = v.y; out[2] = v.z; out[3] = v.w;
        } else {
            const double2 v0 = *reinterpret_cast<const double2*>(col + rb);
            const double2 v1 = *reinterpret_cast<const double2*>(col + rb + 2);
            out[0] = v0.x; out[1] = v0.y; out[2] = v1.x; out[3] = v1.y;
        }
    } else {
#pragma unroll
        for (int i = 0; i < 4; ++i) out[i] = rb + i < NE ? col[rb + i] : T(0);
    }
}

template <typename T> __device__ __forceinline__ void store_rows4(T* col, int rb, int NE, bool v4, const T* v) {
    if (rb >= NE) return;
    if (v4) {
        if constexpr (sizeof(T) == 4) {
            *reinterpret_cast<float4*>(col + rb) = make_float4(v[0], v[1], v[2], v[3]);
        } else {
            *reinterpret_cast<double2*>(col + rb) = make_double2(v[0], v[1]);
            *reinterpret_cast<double2*>(col + rb + 2) = make_double2(v[2], v[3]);
        }
    } else {
#pragma unroll
        for (int i = 0; i < 4; ++i)
            if (rb + i < NE) col[rb + i] = v[i];
    }
}

// four consecutive LDS values at a 4-aligned offset of a 16-byte aligned array
template <typename T> __device__ __forceinline__ void lds_rows4(const T* p, T* out) {
    if constexpr (sizeof(T) == 4) {
        const float4 v = *reinterpret_cast<const float4*>(p);
        out[0] = v.x; out[1] = v.y; out[2] = v.z; out[3] = v.w;
    } else {
        const double2 v0 = *reinterpret_cast<const double2*>(p);
        const double2 v1 = *reinterpret_cast<const double2*>(p + 2);
        out[0] = v0.x; out[1] = v0.y; out[2] = v1.x; out[3] = v1.y;
    }
}

// TO: storage of S^-1.  For FP16 storage (T = float) the working matrix cannot live in the output
// block; the element's K slot (NE^2 doubles) then holds K converted to FP32 in its first half and
// the working matrix in its second half, and only the final permuted store writes the output.
template <typename T, typename TO, int RR, int PB>
__global__ void __launch_bounds__(BIG_THREADS) bj_invert_big_kernel(double* KT, const double* __restrict__ HT,
                                                                   TO* __restrict__ SinvT, int NE,
                                                                   T a1dt, T bc, int* __restrict__ status) {
    constexpr bool HALF = sizeof(TO) == 2;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const BigLds<T> L = big_lds<T>(NE, PB);
    const int nep = L.nep;
    T* sP = reinterpret_cast<T*>(smem_raw);                      // panel: sP[j * nep + r]
    T* sA = sP;                                                  // K^2 staging: sA[t * 64 + x]
    T* sB = sP + BIG_KC * BIG_TILE;                              //              sB[t * 65 + y]
    T* sU = reinterpret_cast<T*>(smem_raw + L.off_u);            // sU[j * 64 + y]
    T* s_col = reinterpret_cast<T*>(smem_raw + L.off_col);
    T* s_row = reinterpret_cast<T*>(smem_raw + L.off_row);
    int* s_ired = reinterpret_cast<int*>(smem_raw + L.off_ired);
    int* s_prow = reinterpret_cast<int*>(smem_raw + L.off_prow); // pivot row of step k
    int* s_pinv = reinterpret_cast<int*>(smem_raw + L.off_pinv); // step at which row r was pivot, or -1

    const int tid = threadIdx.x;
    const int tr = tid % 16, tc = tid / 16;
    const size_t e = blockIdx.x;
    const size_t nn = (size_t)NE * NE;
    double* Kd = KT + e * nn;
    float* Kf = reinterpret_cast<float*>(Kd);                   // HALF: FP32 copy of K, first half of the slot
    T* A = HALF ? reinterpret_cast<T*>(Kf + nn) : reinterpret_cast<T*>(SinvT + e * nn);
    auto Kat = [&](size_t i) -> double { return HALF ? (double)Kf[i] : Kd[i]; };
    if constexpr (HALF) {
        // in place, chunk by chunk: the floats of chunk c overwrite doubles of chunks <= c, which
        // have been read (each chunk's loads finish at the barrier before its stores)
        constexpr int CH = 4 * BIG_THREADS;
        for (size_t c0 = 0; c0 < nn; c0 += CH) {
            double v[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const size_t i = c0 + tid + (size_t)q * BIG_THREADS;
                v[q] = i < nn ? Kd[i] : 0.0;
            }
            __syncthreads();
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const size_t i = c0 + tid + (size_t)q * BIG_THREADS;
                if (i < nn) Kf[i] = (float)v[q];
            }
            __syncthreads();
        }
    }

    // ---- S = I - a1dt K + bc (K^2 + H) into A (K staged through LDS in slabs of 16, the next slab's
    // loads issued before the current slab's products)
    {
        const int xa = tid % BIG_TILE, ta = tid / BIG_TILE;   // sA: t = ta + 4 q, x = xa
        const int yb = tid / BIG_KC, tb = tid % BIG_KC;       // sB: y = yb + 16 q, t = tb
        for (int r0 = 0; r0 < NE; r0 += BIG_TILE)
            for (int c0 = 0; c0 < NE; c0 += BIG_TILE) {
                T acc[4][4];
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int b = 0; b < 4; ++b) acc[i][b] = T(0);
                double ga[4], gb[4];
                auto fetch = [&](int kk) {
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int k = kk + ta + 4 * q, r = r0 + xa;
                        ga[q] = (k < NE && r < NE) ? Kat((size_t)k * NE + r) : 0.0;       // K[r][k]
                        const int k2 = kk + tb, cc = c0 + yb + 16 * q;
                        gb[q] = (k2 < NE && cc < NE) ? Kat((size_t)cc * NE + k2) : 0.0;   // K[k][c]
                    }
                };
                fetch(0);
                for (int kk = 0; kk < NE; kk += BIG_KC) {
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        sA[(ta + 4 * q) * BIG_TILE + xa] = (T)ga[q];
                        sB[tb * (BIG_TILE + 1) + yb + 16 * q] = (T)gb[q];
                    }
                    __syncthreads();
                    if (kk + BIG_KC < NE) fetch(kk + BIG_KC);
#pragma unroll 4
                    for (int t = 0; t < BIG_KC; ++t) {
                        T ra[4], cb[4];
#pragma unroll
                        for (int i = 0; i < 4; ++i) ra[i] = sA[t * BIG_TILE + 4 * tr + i];
#pragma unroll
                        for (int b = 0; b < 4; ++b) cb[b] = sB[t * (BIG_TILE + 1) + tc + 16 * b];
#pragma unroll
                        for (int i = 0; i < 4; ++i)
#pragma unroll
                            for (int b = 0; b < 4; ++b) acc[i][b] += ra[i] * cb[b];
                    }
                    __syncthreads();
                }
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    const int cc = c0 + tc + 16 * b;
                    if (cc >= NE) continue;
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int r = r0 + 4 * tr + i;
                        if (r >= NE) continue;
                        T v = (r == cc) ? T(1) : T(0);
                        const T h = HT ? (T)HT[e * nn + (size_t)cc * NE + r] : T(0);
                        v += -a1dt * (T)Kat((size_t)cc * NE + r) + bc * (acc[i][b] + h);
                        A[(size_t)cc * NE + r] = v;
                    }
                }
            }
    }
    for (int r = tid; r < NE; r += BIG_THREADS) s_pinv[r] = -1;
    __syncthreads();

    const bool v4 = (NE % 4) == 0;   // 4 consecutive rows of a column: one aligned 4-value access
    // ---- panels.  Panel phase in registers: lane pr of wave pc owns rows pr + 64 a (a < RR) and
    // panel columns pc + 4 b (b < RC), so one wave holds whole columns and finds a pivot alone.
    constexpr int RC = PB / 4;
    const int pr = tid & 63, pc = tid >> 6;
    unsigned used = 0u;   // bit a: owned row pr + 64 a has been a pivot row (any panel)
    for (int k0 = 0; k0 < NE; k0 += PB) {
        const int pb = NE - k0 < PB ? NE - k0 : PB;
        T P[RR][RC];
#pragma unroll
        for (int b = 0; b < RC; ++b) {
            const int jj = pc + 4 * b;
#pragma unroll
            for (int a = 0; a < RR; ++a) {
                const int r = pr + 64 * a;
                P[a][b] = (r < NE && jj < pb) ? A[(size_t)(k0 + jj) * NE + r] : T(0);
            }
        }
        for (int j = 0; j < pb; ++j) {
            const int k = k0 + j;
            const int bk = j >> 2;
            if (pc == (j & 3)) {           // pivot: largest |entry| of column j over rows not yet pivot
                T best = T(-1);            // (NaN never wins; smallest row on ties)
                int bi = NE;
#pragma unroll
                for (int a = 0; a < RR; ++a) {
                    const int r = pr + 64 * a;
                    T v = T(0);
#pragma unroll
                    for (int b = 0; b < RC; ++b) v = (b == bk) ? P[a][b] : v;
                    v = v >= T(0) ? v : -v;
                    const bool take = r < NE && !((used >> a) & 1u) && v > best;
                    best = take ? v : best;
                    bi = take ? r : bi;
                }
                wave_argmax(best, bi);
                if (pr == 0) s_ired[0] = bi;
            }
            __syncthreads();
            const int p = s_ired[0];
            if (p >= NE) {                 // no finite pivot left: flag, stop
                if (tid == 0) atomicOr(status, 1);
                return;
            }
            const int ap = p >> 6;
            if (pr == (p & 63)) {          // owners of row p publish it
                used |= 1u << ap;
#pragma unroll
                for (int b = 0; b < RC; ++b) {
                    T v = T(0);
#pragma unroll
                    for (int a = 0; a < RR; ++a) v = (a == ap) ? P[a][b] : v;
                    if (pc + 4 * b < pb) s_row[pc + 4 * b] = v;
                }
            }
            if (pc == (j & 3)) {           // owners of column j publish it
#pragma unroll
                for (int a = 0; a < RR; ++a) {
                    const int r = pr + 64 * a;
                    T v = T(0);
#pragma unroll
                    for (int b = 0; b < RC; ++b) v = (b == bk) ? P[a][b] : v;
                    if (r < NE) s_col[r] = v;
                }
            }
            if (tid == 0) {
                s_prow[k] = p;
                s_pinv[p] = k;
            }
            __syncthreads();
            const T piv = s_col[p];
            const T ipiv = T(1) / piv;
            if (tid == 0 && (!(piv == piv) || piv == T(0))) atomicOr(status, 1);
            T prv[RC], f[RR];
#pragma unroll
            for (int b = 0; b < RC; ++b) prv[b] = pc + 4 * b < pb ? s_row[pc + 4 * b] * ipiv : T(0);
#pragma unroll
            for (int a = 0; a < RR; ++a) f[a] = pr + 64 * a < NE ? s_col[pr + 64 * a] : T(0);
            // exchange step, branch-free: pivot row / pivot column / the rest
#pragma unroll
            for (int a = 0; a < RR; ++a) {
                const bool isp = (pr + 64 * a == p);
                const T pk = isp ? ipiv : -f[a] * ipiv;
#pragma unroll
                for (int b = 0; b < RC; ++b) {
                    const bool isk = (pc + 4 * b == j);
                    const T v = isp ? prv[b] : P[a][b] - f[a] * prv[b];
                    P[a][b] = isk ? pk : v;
                }
            }
        }
        // the eliminated panel: to LDS (the update's left factor) and back to its columns of A
#pragma unroll
        for (int b = 0; b < RC; ++b) {
            const int jj = pc + 4 * b;
            if (jj >= pb) continue;
#pragma unroll
            for (int a = 0; a < RR; ++a) {
                const int r = pr + 64 * a;
                if (r < NE) {
                    sP[jj * nep + r] = P[a][b];
                    A[(size_t)(k0 + jj) * NE + r] = P[a][b];
                }
            }
        }
        __syncthreads();
        // block exchange on the columns outside the panel
        for (int c0 = 0; c0 < NE; c0 += BIG_TILE) {
            for (int i = tid; i < pb * BIG_TILE; i += BIG_THREADS) {
                const int j = i / BIG_TILE, y = i % BIG_TILE;
                const int cc = c0 + y;
                sU[j * BIG_TILE + y] = cc < NE ? A[(size_t)cc * NE + s_prow[k0 + j]] : T(0);
            }
            __syncthreads();
            for (int r0 = 0; r0 < NE; r0 += BIG_TILE) {
                const int rb = r0 + 4 * tr;
                T base[4][4], acc[4][4];
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    const int cc = c0 + tc + 16 * b;
                    load_rows4(A + (size_t)cc * NE, rb, NE, cc < NE, v4, base[b]);
#pragma unroll
                    for (int i = 0; i < 4; ++i) acc[b][i] = T(0);
                }
                if (rb < nep) {
                    for (int j = 0; j < pb; ++j) {
                        T ra[4], cb[4];
                        lds_rows4(sP + j * nep + rb, ra);
#pragma unroll
                        for (int b = 0; b < 4; ++b) cb[b] = sU[j * BIG_TILE + tc + 16 * b];
#pragma unroll
                        for (int b = 0; b < 4; ++b)
#pragma unroll
                            for (int i = 0; i < 4; ++i) acc[b][i] += ra[i] * cb[b];
                    }
                }
                bool inp[4];   // pivot rows of this panel: B^-1 U replaces the row
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int q = rb + i < NE ? s_pinv[rb + i] : -1;
                    inp[i] = q >= k0 && q < k0 + pb;
                }
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    const int cc = c0 + tc + 16 * b;
                    if (cc >= NE || (cc >= k0 && cc < k0 + pb)) continue;
                    T out[4];
#pragma unroll
                    for (int i = 0; i < 4; ++i) out[i] = inp[i] ? acc[b][i] : base[b][i] + acc[b][i];
                    store_rows4(A + (size_t)cc * NE, rb, NE, v4, out);
                }
            }
            __syncthreads();
        }
    }
    // ---- S^-1[pinv[r]][prow[c]] = A[r][c], stored column-major (SinvT[col][row])
    TO* out = SinvT + e * nn;
    if constexpr (HALF) {   // A is in the K slot: one permuted, rounded store (out-of-range entries flagged)
        for (size_t i = tid; i < nn; i += BIG_THREADS) {
            const int cc = (int)(i / NE), r = (int)(i % NE);
            const T v = A[i];
            if (!(v <= T(65504) && v >= T(-65504))) atomicOr(status, 1);
            out[(size_t)s_prow[cc] * NE + s_pinv[r]] = (TO)v;
        }
    } else {                // A is the output block: copy it to the K slot first
        T* slot = reinterpret_cast<T*>(KT + e * nn);
        for (size_t i = tid; i < nn; i += BIG_THREADS) slot[i] = A[i];
        __syncthreads();
        for (size_t i = tid; i < nn; i += BIG_THREADS) {
            const int cc = (int)(i / NE), r = (int)(i % NE);
            out[(size_t)s_prow[cc] * NE + s_pinv[r]] = (TO)slot[i];
        }
    }
}

// the arithmetic follows the storage of S^-1: FP64 blocks are formed and inverted in FP64, FP32
// blocks (mixed precision) in FP32 from the FP64 K; FP16 blocks in FP32, rounded once when stored
template <int TGR, int TGC, int RR, int RC, typename TO>
static hipError_t launch_inv(const double* KT, const double* HT, TO* SinvT, int NE, int nE, double a1dt, double bc, int* status,
                             hipStream_t st) {
    using T = typename std::conditional<sizeof(TO) == 2, float, TO>::type;
    hipLaunchKernelGGL((bj_invert_kernel<TGR, TGC, RR, RC, T, TO>), dim3(nE), dim3(TGR * TGC), 0, st, KT, HT, SinvT,
                       NE, (T)a1dt, (T)bc, status);
    return hipGetLastError();
}

// blocked kernel configurations: rows per lane RR (NE <= 64 RR) and panel width PB, chosen so that
// the panel fits in registers and its LDS copy (PB x NE) in 64 KiB
template <typename TO, int RR, int PB>
static hipError_t launch_big(double* KT, const double* HT, TO* SinvT, int NE, int nE, double a1dt, double bc, int* status,
                             hipStream_t st) {
    using T = typename std::conditional<sizeof(TO) == 2, float, TO>::type;
    const size_t sh = big_lds<T>(NE, PB).bytes;
    if (sh > 65536) return hipErrorInvalidValue;
    hipLaunchKernelGGL((bj_invert_big_kernel<T, TO, RR, PB>), dim3(nE), dim3(BIG_THREADS), sh, st, KT, HT, SinvT, NE,
                       (T)a1dt, (T)bc, status);
    return hipGetLastError();
}

template <typename T>
static hipError_t launch_inv_big(double* KT, const double* HT, T* SinvT, int NE, int nE, double a1dt, double bc, int* status,
                                 hipStream_t st) {
    constexpr bool F = sizeof(T) <= 4;   // FP32 arithmetic (FP32 or FP16 storage)
    if (NE <= 320) return launch_big<T, 5, F ? 32 : 16>(KT, HT, SinvT, NE, nE, a1dt, bc, status, st);
    if (NE <= 640) return launch_big<T, 10, F ? 16 : 8>(KT, HT, SinvT, NE, nE, a1dt, bc, status, st);
    if (NE <= 1024) return launch_big<T, 16, F ? 8 : 4>(KT, HT, SinvT, NE, nE, a1dt, bc, status, st);
    return hipErrorInvalidValue;
}

// KT: the chunk's K blocks; for blocks above 144 unknowns they are overwritten (used as scratch).
// HT: the chunk's Hessian blocks H (BJ^H_ext), same layout, or nullptr (BJ_ext).
// type: storage of S^-1, 0 FP64, 1 FP32, 2 FP16
hipError_t bj_invert(double* KT, const double* HT, void* SinvT, int type, int NE, int nE, double a1dt, double bc, int* status,
                     hipStream_t st) {
    if (nE == 0) return hipSuccess;
    if (NE > 144 && NE <= 1024) {
        if (type == 2) return launch_inv_big<_Float16>(KT, HT, (_Float16*)SinvT, NE, nE, a1dt, bc, status, st);
        return type == 1 ? launch_inv_big<float>(KT, HT, (float*)SinvT, NE, nE, a1dt, bc, status, st)
                         : launch_inv_big<double>(KT, HT, (double*)SinvT, NE, nE, a1dt, bc, status, st);
    }
    if (NE > 144) return hipErrorInvalidValue;
#define HBPC_INV(TGR, TGC, RR, RC)                                                                         \
    if (type == 2) return launch_inv<TGR, TGC, RR, RC, _Float16>(KT, HT, (_Float16*)SinvT, NE, nE, a1dt, bc, status, st); \
    return type == 1 ? launch_inv<TGR, TGC, RR, RC, float>(KT, HT, (float*)SinvT, NE, nE, a1dt, bc, status, st)    \
                     : launch_inv<TGR, TGC, RR, RC, double>(KT, HT, (double*)SinvT, NE, nE, a1dt, bc, status, st);
    if (NE <= 16) { HBPC_INV(4, 4, 4, 4) }
    if (NE <= 32) { HBPC_INV(8, 8, 4, 4) }
    if (NE <= 64) { HBPC_INV(16, 16, 4, 4) }
    if (NE <= 144) { HBPC_INV(16, 32, 9, 5) }
#undef HBPC_INV
    return hipErrorInvalidValue;
}
