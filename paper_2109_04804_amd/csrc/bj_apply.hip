// BJ_ext preconditioner apply (Sec. 3.2.3).
//
// The local products K vs and K (vw - a1dt vs) come from the PCPRE operator
// kernel (a = vw - bcoef K vs, c = vs + K (vw - a1dt vs)); since S_i is a
// polynomial in K_i, S^-1 commutes with K and
//   P^-1 (vw, vs) = (D vw + E vs, F vw + G vs) = (S^-1 a, S^-1 c),
// one pass over the stored S^-1 blocks for both right-hand sides.
#include <hip/hip_runtime.h>
#include <cstdint>

// y = S^-1 x for the two right-hand sides (w block, sigma block).
// yw = S^-1 xa, ys = S^-1 xc per element; S^-1 stored transposed (column-major blocks, SinvT[e][c][r]),
// each thread owns groups of VR consecutive rows (one 16-byte load per column when VR * sizeof(TM)
// == 16): min(NE / VR, 256) threads per element, a thread taking every tpe-th group when there are
// more groups than threads; several elements per block; the two right-hand sides staged in LDS
template <typename TM, typename T, int VR>
__global__ void __launch_bounds__(256) bj_apply_kernel(const TM* __restrict__ SinvT, const T* __restrict__ xa,
                                                      const T* __restrict__ xc, T* __restrict__ yw,
                                                      T* __restrict__ ys, int NE, int nE) {
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
        sx[2 * i] = ok ? xa[g] : T(0);
        sx[2 * i + 1] = ok ? xc[g] : T(0);
    }
    __syncthreads();
    const int e = e0 + el;
    if (el >= epb || e >= nE) return;
    typedef TM VT __attribute__((ext_vector_type(VR)));
    const T* x = sx + 2 * el * NE;
    for (int gr = threadIdx.x % tpe; gr < ng; gr += tpe) {
        const int r0 = gr * VR;
        const TM* M = SinvT + (size_t)e * NE * NE + r0;
        T s0[VR], s1[VR];
#pragma unroll
        for (int q = 0; q < VR; ++q) s0[q] = s1[q] = T(0);
#pragma unroll 4
        for (int c = 0; c < NE; ++c) {
            const VT m = *reinterpret_cast<const VT*>(M + (size_t)c * NE);
            const T xa_c = x[2 * c], xc_c = x[2 * c + 1];
#pragma unroll
            for (int q = 0; q < VR; ++q) {
                s0[q] += (T)m[q] * xa_c;
                s1[q] += (T)m[q] * xc_c;
            }
        }
#pragma unroll
        for (int q = 0; q < VR; ++q) {
            yw[(size_t)e * NE + r0 + q] = s0[q];
            ys[(size_t)e * NE + r0 + q] = s1[q];
        }
    }
}

template <typename TM, typename T, int VR>
static void launch_apply(const TM* SinvT, const T* xa, const T* xc, T* yw, T* ys, int NE, int nE, hipStream_t st) {
    const int ng = NE / VR;
    const int tpe = ng < 256 ? ng : 256;
    const int epb = 256 / tpe;
    const int threads = epb * tpe;
    const int grid = (nE + epb - 1) / epb;
    const size_t sh = (size_t)2 * epb * NE * sizeof(T);
    hipLaunchKernelGGL((bj_apply_kernel<TM, T, VR>), dim3(grid), dim3(threads), sh, st, SinvT, xa, xc, yw, ys, NE, nE);
}

// rows per thread: a 16-byte load of S^-1 when NE allows it
template <typename TM, typename T>
static void apply_vr(const void* SinvT, const void* xa, const void* xc, void* yw, void* ys, int NE, int nE,
                     hipStream_t st) {
    constexpr int V = 16 / sizeof(TM);
    const TM* M = (const TM*)SinvT;
    if (NE % V == 0)
        launch_apply<TM, T, V>(M, (const T*)xa, (const T*)xc, (T*)yw, (T*)ys, NE, nE, st);
    else if (NE % 2 == 0)
        launch_apply<TM, T, 2>(M, (const T*)xa, (const T*)xc, (T*)yw, (T*)ys, NE, nE, st);
    else
        launch_apply<TM, T, 1>(M, (const T*)xa, (const T*)xc, (T*)yw, (T*)ys, NE, nE, st);
}

// m_type: storage of S^-1, 0 FP64, 1 FP32, 2 FP16 (FP32 vectors only); the sums run in the vector type
hipError_t bj_apply(const void* SinvT, int m_type, const void* xa, const void* xc, void* yw, void* ys, int v_f32,
                    int NE, int nE, hipStream_t st) {
    if (nE == 0) return hipSuccess;
    if (NE > 1024) return hipErrorInvalidValue;
    if (m_type == 2 && !v_f32) return hipErrorInvalidValue;
    if (v_f32) {
        if (m_type == 2) apply_vr<_Float16, float>(SinvT, xa, xc, yw, ys, NE, nE, st);
        else if (m_type == 1) apply_vr<float, float>(SinvT, xa, xc, yw, ys, NE, nE, st);
        else apply_vr<double, float>(SinvT, xa, xc, yw, ys, NE, nE, st);
    } else {
        if (m_type == 1) apply_vr<float, double>(SinvT, xa, xc, yw, ys, NE, nE, st);
        else apply_vr<double, double>(SinvT, xa, xc, yw, ys, NE, nE, st);
    }
    return hipGetLastError();
}
