// BJ_ext preconditioner apply (Sec. 3.2.3).
//
// The local products K vs and K (vw - a1dt vs) come from the PCPRE operator
// kernel (a = vw - bcoef K vs, c = vs + K (vw - a1dt vs)); since S_i is a
// polynomial in K_i, S^-1 commutes with K and
//   P^-1 (vw, vs) = (D vw + E vs, F vw + G vs) = (S^-1 a, S^-1 c),
// one pass over the stored S^-1 blocks for both right-hand sides.
#include <hip/hip_runtime.h>
#include <cstdint>

// y_k = S^-1 x_k for NR right-hand sides: the w and sigma blocks of one Krylov vector (NR = 2), or
// of two systems that share the blocks (NR = 4: the corrector stages of a sweep solved together).
// S^-1 stored transposed (column-major blocks, SinvT[e][c][r]), each thread owns groups of VR
// consecutive rows (loads of at most 16 bytes, VR * sizeof(TM) bytes per column): min(NE / VR, 256)
// threads per element, a thread taking every tpe-th group when there are more groups than threads;
// several elements per block; the right-hand sides staged in LDS.  One pass over S^-1 serves all NR.
template <typename T, int NR> struct ApplyVecs {
    const T* x[NR];
    T* y[NR];
};

template <typename TM, typename T, int VR, int NR, int UNR>
__global__ void __launch_bounds__(256) bj_apply_kernel(const TM* __restrict__ SinvT, ApplyVecs<T, NR> v, int NE,
                                                      int nE) {
    extern __shared__ unsigned char smem_raw[];
    T* sx = reinterpret_cast<T*>(smem_raw);
    const int ng = NE / VR;
    const int tpe = ng < 256 ? ng : 256;
    const int epb = blockDim.x / tpe;
    const int el = threadIdx.x / tpe;
    const int e0 = blockIdx.x * epb;
    for (int i = threadIdx.x; i < epb * NE; i += blockDim.x) {
        int le = i / NE;
        size_t g = (size_t)(e0 + le) * NE + (i % NE);
        bool ok = e0 + le < nE;
#pragma unroll
        for (int k = 0; k < NR; ++k) sx[NR * i + k] = ok ? v.x[k][g] : T(0);
    }
    __syncthreads();
    const int e = e0 + el;
    if (el >= epb || e >= nE) return;
    constexpr int LV = 16 / sizeof(TM) < VR ? 16 / (int)sizeof(TM) : VR;   // values per load (<= 16 bytes)
    typedef TM VT __attribute__((ext_vector_type(LV)));
    const T* x = sx + NR * el * NE;
    for (int gr = threadIdx.x % tpe; gr < ng; gr += tpe) {
        const int r0 = gr * VR;
        const TM* M = SinvT + (size_t)e * NE * NE + r0;
        T s[NR][VR];
#pragma unroll
        for (int k = 0; k < NR; ++k)
#pragma unroll
            for (int q = 0; q < VR; ++q) s[k][q] = T(0);
#pragma unroll UNR
        for (int c = 0; c < NE; ++c) {
            TM m[VR];
#pragma unroll
            for (int h = 0; h < VR / LV; ++h) {
                const VT t = *reinterpret_cast<const VT*>(M + (size_t)c * NE + h * LV);
#pragma unroll
                for (int q = 0; q < LV; ++q) m[h * LV + q] = t[q];
            }
#pragma unroll
            for (int k = 0; k < NR; ++k) {
                const T xc = x[NR * c + k];
#pragma unroll
                for (int q = 0; q < VR; ++q) s[k][q] += (T)m[q] * xc;
            }
        }
#pragma unroll
        for (int k = 0; k < NR; ++k)
#pragma unroll
            for (int q = 0; q < VR; ++q) v.y[k][(size_t)e * NE + r0 + q] = s[k][q];
    }
}

template <typename TM, typename T, int VR, int NR, int UNR = 4>
static void launch_apply(const TM* SinvT, const ApplyVecs<T, NR>& v, int NE, int nE, hipStream_t st) {
    const int ng = NE / VR;
    const int tpe = ng < 256 ? ng : 256;
    const int epb = 256 / tpe;
    const int threads = epb * tpe;
    const int grid = (nE + epb - 1) / epb;
    const size_t sh = (size_t)NR * epb * NE * sizeof(T);
    hipLaunchKernelGGL((bj_apply_kernel<TM, T, VR, NR, UNR>), dim3(grid), dim3(threads), sh, st, SinvT, v, NE, nE);
}

// rows per thread: a 16-byte load of S^-1 when NE allows it
template <typename TM, typename T, int NR>
static void apply_vr(const void* SinvT, const void* const* xs, void* const* ys, int NE, int nE, hipStream_t st) {
    constexpr int V = 16 / sizeof(TM);
    const TM* M = (const TM*)SinvT;
    ApplyVecs<T, NR> v;
    for (int k = 0; k < NR; ++k) {
        v.x[k] = (const T*)xs[k];
        v.y[k] = (T*)ys[k];
    }
    if constexpr (sizeof(TM) == 4 && sizeof(T) == 4) {
        // FP32 blocks and vectors: rows per thread and unroll depth as measured fastest for the
        // element blocks of the 2-D (NE = 144) and 3-D (NE = 320) Euler workloads, each with two
        // and four right-hand sides (the others keep 4 rows and an unroll of 4)
        if (NE <= 160) {
            if (NR == 2 && NE % 8 == 0) return launch_apply<TM, T, 8, NR, 4>(M, v, NE, nE, st);
            if (NR == 4 && NE % 4 == 0) return launch_apply<TM, T, 4, NR, 2>(M, v, NE, nE, st);
        } else {
            if (NR == 2 && NE % 4 == 0) return launch_apply<TM, T, 4, NR, 8>(M, v, NE, nE, st);
            if (NR == 4 && NE % 8 == 0) return launch_apply<TM, T, 8, NR, 2>(M, v, NE, nE, st);
        }
    }
    if (NE % V == 0)
        launch_apply<TM, T, V, NR>(M, v, NE, nE, st);
    else if (NE % 2 == 0)
        launch_apply<TM, T, 2, NR>(M, v, NE, nE, st);
    else
        launch_apply<TM, T, 1, NR>(M, v, NE, nE, st);
}

template <typename TM, typename T>
static void apply_nr(const void* SinvT, const void* const* xs, void* const* ys, int nr, int NE, int nE,
                     hipStream_t st) {
    if (nr == 4) apply_vr<TM, T, 4>(SinvT, xs, ys, NE, nE, st);
    else apply_vr<TM, T, 2>(SinvT, xs, ys, NE, nE, st);
}

// y_k = S^-1 x_k, k < nr (2 or 4); m_type: storage of S^-1, 0 FP64, 1 FP32, 2 FP16 (FP32 vectors only)
hipError_t bj_apply_n(const void* SinvT, int m_type, const void* const* xs, void* const* ys, int nr, int v_f32,
                      int NE, int nE, hipStream_t st) {
    if (nE == 0) return hipSuccess;
    if (NE > 1024 || (nr != 2 && nr != 4)) return hipErrorInvalidValue;
    if (m_type == 2 && !v_f32) return hipErrorInvalidValue;
    if (v_f32) {
        if (m_type == 2) apply_nr<_Float16, float>(SinvT, xs, ys, nr, NE, nE, st);
        else if (m_type == 1) apply_nr<float, float>(SinvT, xs, ys, nr, NE, nE, st);
        else apply_nr<double, float>(SinvT, xs, ys, nr, NE, nE, st);
    } else {
        if (m_type == 1) apply_nr<float, double>(SinvT, xs, ys, nr, NE, nE, st);
        else apply_nr<double, double>(SinvT, xs, ys, nr, NE, nE, st);
    }
    return hipGetLastError();
}

// the two right-hand sides of one Krylov vector; the sums run in the vector type
hipError_t bj_apply(const void* SinvT, int m_type, const void* xa, const void* xc, void* yw, void* ys, int v_f32,
                    int NE, int nE, hipStream_t st) {
    const void* xs[2] = {xa, xc};
    void* ys2[2] = {yw, ys};
    return bj_apply_n(SinvT, m_type, xs, ys2, 2, v_f32, NE, nE, st);
}
