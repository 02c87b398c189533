// Vector kernels of the Newton-Krylov solver: block-partial dot products with
// several basis vectors at once (classical Gram-Schmidt, twice, the second
// pass from the Gram matrix of the basis), the update w -= V h with the normalisation of w,
// axpby, casts.  Reductions are deterministic: each block sums
// a fixed set of indices in a fixed order, partial results are combined by
// one block in a fixed tree, so two runs give bitwise equal results.
#include <hip/hip_runtime.h>
#include <type_traits>
#include <algorithm>
#include <cstddef>
#include <cstdint>

constexpr int BLAS_THREADS = 256;
constexpr int MDOT_CHUNK = 16;
constexpr int MDOT2_CHUNK = 16;
// most basis vectors of one Gram-Schmidt pass (the FGMRES restart length)
constexpr int GS_MAXK = 1024;

template <typename T> __device__ __forceinline__ double block_sum(double v, double* sh) {
    // wave64 shuffle tree, then LDS across the 4 waves
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0) {
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) r += sh[i];
    }
    return r;
}

// Grid-wide "last block" hand-over: every block publishes its result, then takes a ticket; the
// block with the last ticket sees every published result (device-scope fences around the ticket)
// and finishes the reduction, then rewinds the counter for the next launch.
__device__ __forceinline__ bool last_block(unsigned* counter, unsigned nblocks) {
    __shared__ bool last;
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        last = atomicAdd(counter, 1u) == nblocks - 1;
    }
    __syncthreads();
    if (last) __threadfence();
    return last;
}

// VEC consecutive values of type T as one 16-byte (or scalar) load/store
template <typename T, int VEC> struct Vec { T v[VEC]; };
template <typename T, int VEC> __device__ __forceinline__ Vec<T, VEC> vload(const T* p) {
    Vec<T, VEC> r;
    if constexpr (VEC == 1) {
        r.v[0] = *p;
    } else {
        typedef T VT __attribute__((ext_vector_type(VEC)));
        const VT x = *reinterpret_cast<const VT*>(p);
#pragma unroll
        for (int i = 0; i < VEC; ++i) r.v[i] = x[i];
    }
    return r;
}
template <typename T, int VEC> __device__ __forceinline__ void vstore(T* p, const Vec<T, VEC>& r) {
    if constexpr (VEC == 1) {
        *p = r.v[0];
    } else {
        typedef T VT __attribute__((ext_vector_type(VEC)));
        VT x;
#pragma unroll
        for (int i = 0; i < VEC; ++i) x[i] = r.v[i];
        *reinterpret_cast<VT*>(p) = x;
    }
}

// part[(c0 + j) * gridDim.x + blockIdx.x] = sum_{i in block} V_j[i] * w[i], j < kc (<= MDOT_CHUNK)
// (block partials column by column, so that the reduction reads them contiguously); VEC values per
// load (n and ld multiples of VEC)
template <typename T, int VEC>
__global__ void __launch_bounds__(BLAS_THREADS) mdot_kernel(const T* __restrict__ V, size_t ld, int kc,
                                                            const T* __restrict__ w, size_t n,
                                                            double* __restrict__ part, int c0) {
    __shared__ double shw[BLAS_THREADS / 64][MDOT_CHUNK];
    double acc[MDOT_CHUNK];
#pragma unroll
    for (int j = 0; j < MDOT_CHUNK; ++j) acc[j] = 0.0;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    const size_t nv = n / VEC;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < nv; i += stride) {
        const Vec<T, VEC> wv = vload<T, VEC>(w + i * VEC);
#pragma unroll
        for (int j = 0; j < MDOT_CHUNK; ++j)
            if (j < kc) {
                const Vec<T, VEC> vv = vload<T, VEC>(V + j * ld + i * VEC);
                double s = 0.0;
#pragma unroll
                for (int q = 0; q < VEC; ++q) s += (double)vv.v[q] * (double)wv.v[q];
                acc[j] += s;
            }
    }
    // all kc sums at once: wave shuffle trees, then one LDS exchange across the waves
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int j = 0; j < MDOT_CHUNK; ++j) {
        if (j < kc) {
            double v = acc[j];
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
            if (lane == 0) shw[wid][j] = v;
        }
    }
    __syncthreads();
    if (threadIdx.x < kc) {
        double r = 0.0;
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) r += shw[i][threadIdx.x];
        part[(size_t)(c0 + threadIdx.x) * gridDim.x + blockIdx.x] = r;
    }
}

// column c0 + j of the block partials (layout as for mdot_kernel): sum V_j[i] w1[i]; column
// off2 + c0 + j: sum V_j[i] w2[i], for j < kc (<= MDOT2_CHUNK): the projections of a new vector and
// the Gram column of the newest basis vector in one pass over V.  blockIdx.y selects the system
// (g0, or g1 for the second system of a pair of stage solves); kc = 0: no work for it.
template <typename T> struct GramSys {
    const T* V;
    const T* w1;
    const T* w2;
    double* part;
    int kc, c0, off2;
};

template <typename T, int VEC>
__global__ void __launch_bounds__(BLAS_THREADS) mdot2_kernel(GramSys<T> g0, GramSys<T> g1, size_t ld, size_t n) {
    const GramSys<T>& g = blockIdx.y ? g1 : g0;
    const int kc = g.kc;
    if (kc <= 0) return;
    const T* __restrict__ V = g.V;
    const T* __restrict__ w1 = g.w1;
    const T* __restrict__ w2 = g.w2;
    __shared__ double shw[BLAS_THREADS / 64][2 * MDOT2_CHUNK];
    double a1[MDOT2_CHUNK], a2[MDOT2_CHUNK];
#pragma unroll
    for (int j = 0; j < MDOT2_CHUNK; ++j) a1[j] = a2[j] = 0.0;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    const size_t nv = n / VEC;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < nv; i += stride) {
        const Vec<T, VEC> x1 = vload<T, VEC>(w1 + i * VEC);
        const Vec<T, VEC> x2 = vload<T, VEC>(w2 + i * VEC);
#pragma unroll
        for (int j = 0; j < MDOT2_CHUNK; ++j)
            if (j < kc) {
                const Vec<T, VEC> vv = vload<T, VEC>(V + j * ld + i * VEC);
                double s1 = 0.0, s2 = 0.0;
#pragma unroll
                for (int q = 0; q < VEC; ++q) {
                    s1 += (double)vv.v[q] * (double)x1.v[q];
                    s2 += (double)vv.v[q] * (double)x2.v[q];
                }
                a1[j] += s1;
                a2[j] += s2;
            }
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int j = 0; j < MDOT2_CHUNK; ++j) {
        if (j < kc) {
            double v1 = a1[j], v2 = a2[j];
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) {
                v1 += __shfl_down(v1, off, 64);
                v2 += __shfl_down(v2, off, 64);
            }
            if (lane == 0) {
                shw[wid][j] = v1;
                shw[wid][MDOT2_CHUNK + j] = v2;
            }
        }
    }
    __syncthreads();
    if (threadIdx.x < 2 * kc) {
        const int j = threadIdx.x < kc ? threadIdx.x : threadIdx.x - kc + MDOT2_CHUNK;
        double r = 0.0;
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) r += shw[i][j];
        const int col = g.c0 + (threadIdx.x < kc ? threadIdx.x : g.off2 + threadIdx.x - kc);
        g.part[(size_t)col * gridDim.x + blockIdx.x] = r;
    }
}

// out[j] = sum_b part[j * nb + b] for the 2k columns j = blockIdx.x (out = h1 | g); then the last
// block forms the Gram-Schmidt coefficients of both passes: with G = V^T V (column k-1 = g, stored
// symmetric, leading dimension ldg) and h1 = V^T u, the second classical pass V^T (u - V h1) =
// h1 - G h1, so the two passes together subtract V h with h = 2 h1 - G h1.  blockIdx.y selects the
// system; blocks beyond its 2k columns take no part (nor a ticket).
struct RedSys {
    const double* part;
    double* out;
    int k;
    double* G;
    double* h;
    unsigned* counter;
};

__global__ void __launch_bounds__(BLAS_THREADS) reduce_gram_kernel(RedSys r0, RedSys r1, int nb, int ldg) {
    const RedSys& r = blockIdx.y ? r1 : r0;
    const int k = r.k;
    if ((int)blockIdx.x >= 2 * k) return;
    __shared__ double sh[BLAS_THREADS / 64];
    const int j = blockIdx.x;
    double s = 0.0;
    for (int b = threadIdx.x; b < nb; b += blockDim.x) s += r.part[(size_t)j * nb + b];
    s = block_sum<double>(s, sh);
    if (threadIdx.x == 0) r.out[j] = s;
    if (!last_block(r.counter, 2u * k)) return;
    const double* h1 = r.out;
    const double* g = r.out + k;
    double* G = r.G;
    const int jj = k - 1;
    for (int i = threadIdx.x; i <= jj; i += blockDim.x) {
        G[(size_t)i * ldg + jj] = g[i];
        G[(size_t)jj * ldg + i] = g[i];
    }
    __syncthreads();
    for (int i = threadIdx.x; i <= jj; i += blockDim.x) {
        double t = 0.0;
        for (int l = 0; l <= jj; ++l) t += G[(size_t)i * ldg + l] * h1[l];
        r.h[i] = 2.0 * h1[i] - t;
    }
    if (threadIdx.x == 0) *r.counter = 0u;
}

// out[j] = scale * sum_b part[j * nb + b]; one block per j
__global__ void __launch_bounds__(BLAS_THREADS) reduce_parts_kernel(const double* __restrict__ part, int nb,
                                                                    double* __restrict__ out, double scale) {
    __shared__ double sh[BLAS_THREADS / 64];
    const int j = blockIdx.x;
    double s = 0.0;
    for (int b = threadIdx.x; b < nb; b += blockDim.x) s += part[(size_t)j * nb + b];
    s = block_sum<double>(s, sh);
    if (threadIdx.x == 0) out[j] = scale * s;
}

// y[i] = a * x[i] + b * y[i] (b == 0: y is not read)
template <typename TX, typename TY>
__global__ void __launch_bounds__(BLAS_THREADS) axpby_kernel(double a, const TX* x, double b,
                                                             TY* y, size_t n) {   // x may alias y
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        double v = a * (double)x[i];
        if (b != 0.0) v += b * (double)y[i];
        y[i] = (TY)v;
    }
}

// y[i] = a * x[i] + b * z[i]
template <typename T>
__global__ void __launch_bounds__(BLAS_THREADS) lincomb2_kernel(double a, const T* __restrict__ x, double b,
                                                                const T* __restrict__ z, T* __restrict__ y, size_t n) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        y[i] = (T)(a * (double)x[i] + b * (double)z[i]);
}

// y[i] += sum_j c[j] Z_j[i]  (c on the host, passed by value in chunks of 8)
struct Coef8 { double c[8]; };
template <typename TZ, typename TY>
__global__ void __launch_bounds__(BLAS_THREADS) gemv_add_kernel(const TZ* __restrict__ Z, size_t ld, int k, Coef8 c,
                                                                TY* __restrict__ y, size_t n) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        double acc = 0.0;
#pragma unroll
        for (int j = 0; j < 8; ++j)
            if (j < k) acc += c.c[j] * (double)Z[j * ld + i];
        y[i] = (TY)((double)y[i] + acc);
    }
}

// status |= 1 if any non-finite value
template <typename T>
__global__ void __launch_bounds__(BLAS_THREADS) nonfinite_kernel(const T* __restrict__ x, size_t n, int* status) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    int bad = 0;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        T v = x[i];
        if (!(v == v) || v - v != v - v) bad = 1;
    }
    if (bad) atomicOr(status, 1);
}

// ------------------------------------------------------------------ Gram-Schmidt passes
// w[i] -= sum_j h[j] V_j[i] and a per-block partial of ||w||^2 (part[blockIdx.x]); VEC values per
// load (n and ld multiples of VEC).  (A last-block final sum here costs more than a second launch:
// the device-scope release of each block writes back the freshly updated w from L2.)  blockIdx.y
// selects the system (k = 0: none).
template <typename T> struct UpdSys {
    const T* V;
    int k;
    const double* h;
    T* w;
    double* part;
};

template <typename T, int VEC>
__global__ void __launch_bounds__(BLAS_THREADS) gemv_sub_norm_kernel(UpdSys<T> u0, UpdSys<T> u1, size_t ld,
                                                                     size_t n) {
    const UpdSys<T>& u = blockIdx.y ? u1 : u0;
    const int k = u.k;
    if (k <= 0) return;
    const T* __restrict__ V = u.V;
    T* __restrict__ w = u.w;
    __shared__ double sh[GS_MAXK];
    __shared__ double red[BLAS_THREADS / 64];
    for (int j = threadIdx.x; j < k; j += blockDim.x) sh[j] = u.h[j];
    __syncthreads();
    double nrm = 0.0;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    const size_t nv = n / VEC;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < nv; i += stride) {
        double acc[VEC];
#pragma unroll
        for (int q = 0; q < VEC; ++q) acc[q] = 0.0;
        for (int j = 0; j < k; ++j) {
            const Vec<T, VEC> vv = vload<T, VEC>(V + (size_t)j * ld + i * VEC);
            const double hj = sh[j];
#pragma unroll
            for (int q = 0; q < VEC; ++q) acc[q] += hj * (double)vv.v[q];
        }
        Vec<T, VEC> wv = vload<T, VEC>(w + i * VEC);
#pragma unroll
        for (int q = 0; q < VEC; ++q) {
            wv.v[q] = (T)((double)wv.v[q] - acc[q]);
            nrm += (double)wv.v[q] * (double)wv.v[q];
        }
        vstore<T, VEC>(w + i * VEC, wv);
    }
    double t = block_sum<double>(nrm, red);
    if (threadIdx.x == 0) u.part[blockIdx.x] = t;
}

// hn = sum of the nb block partials of ||u||^2 (every block forms the same sum in the same fixed
// order; block 0 stores it in nrm2[0]), then u /= sqrt(hn) (u unchanged when hn is 0);
// blockIdx.y selects the system (null u: none)
template <typename T> struct ScaleSys {
    T* u;
    const double* part;
    double* nrm2;
};

template <typename T>
__global__ void __launch_bounds__(BLAS_THREADS) sum_scale_kernel(ScaleSys<T> s0, ScaleSys<T> s1, size_t n, int nb) {
    const ScaleSys<T>& sc_ = blockIdx.y ? s1 : s0;
    if (!sc_.u) return;
    T* __restrict__ u = sc_.u;
    __shared__ double red[BLAS_THREADS / 64];
    __shared__ double hn_s;
    double s = 0.0;
    for (int b = threadIdx.x; b < nb; b += blockDim.x) s += sc_.part[b];
    s = block_sum<double>(s, red);
    if (threadIdx.x == 0) {
        hn_s = s;
        if (blockIdx.x == 0) sc_.nrm2[0] = s;
    }
    __syncthreads();
    const double hn = hn_s;
    if (!(hn > 0.0)) return;
    const double sc = 1.0 / sqrt(hn);
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) u[i] = (T)(sc * (double)u[i]);
}

// ------------------------------------------------------------------ launchers
static int blas_grid(size_t n, size_t cap = 2048) {
    size_t g = (n + BLAS_THREADS - 1) / BLAS_THREADS;
    if (g > cap) g = cap;
    if (g < 1) g = 1;
    return (int)g;
}

// multi-dot kernels carry many accumulators: fewer, longer-running blocks (4 per CU)
constexpr size_t MDOT_GRID = 1024;

int blas_mdot_grid(size_t n) { return blas_grid(n); }

// 16-byte loads when the vector length, the basis stride and both base addresses allow them
static int vec_of(size_t n, size_t ld, int f32, const void* a, const void* b) {
    const size_t v = f32 ? 4 : 2;
    const bool aligned = ((uintptr_t)a % 16 == 0) && ((uintptr_t)b % 16 == 0);
    return (aligned && n % v == 0 && ld % v == 0) ? (int)v : 1;
}

// h[j] = V_j . w for j < k; part must hold grid * k doubles.
hipError_t blas_mdot(const void* V, size_t ld, int k, const void* w, size_t n, int f32, double* part, double* h,
                     hipStream_t st) {
    const int vec = vec_of(n, ld, f32, V, w);
    int g = blas_grid(n / vec, MDOT_GRID);
    for (int j0 = 0; j0 < k; j0 += MDOT_CHUNK) {
        int kc = k - j0 < MDOT_CHUNK ? k - j0 : MDOT_CHUNK;
        if (f32 && vec == 4)
            hipLaunchKernelGGL((mdot_kernel<float, 4>), dim3(g), dim3(BLAS_THREADS), 0, st,
                               (const float*)V + j0 * ld, ld, kc, (const float*)w, n, part, j0);
        else if (f32)
            hipLaunchKernelGGL((mdot_kernel<float, 1>), dim3(g), dim3(BLAS_THREADS), 0, st,
                               (const float*)V + j0 * ld, ld, kc, (const float*)w, n, part, j0);
        else if (vec == 2)
            hipLaunchKernelGGL((mdot_kernel<double, 2>), dim3(g), dim3(BLAS_THREADS), 0, st,
                               (const double*)V + j0 * ld, ld, kc, (const double*)w, n, part, j0);
        else
            hipLaunchKernelGGL((mdot_kernel<double, 1>), dim3(g), dim3(BLAS_THREADS), 0, st,
                               (const double*)V + j0 * ld, ld, kc, (const double*)w, n, part, j0);
    }
    hipLaunchKernelGGL(reduce_parts_kernel, dim3(k), dim3(BLAS_THREADS), 0, st, part, g, h, 1.0);
    return hipGetLastError();
}

// u -= V h (k columns, h on the device), nrm2[0] = ||u||^2, u /= ||u||: the Arnoldi update of
// a new basis vector.  part: blas_grid(n) doubles.
// For s < ns (1 or 2) systems: u_s -= V_s h_s (k_s columns), then u_s /= ||u_s|| (||u_s||^2 in
// nrm2_s[0]); one launch of each kernel for all systems.  part_s: grid doubles each.
hipError_t blas_gs_update_normalize_n(int ns, const void* const* V, size_t ld, const int* k, const double* const* h,
                                      void* const* u, size_t n, int f32, double* const* part,
                                      double* const* nrm2, hipStream_t st) {
    int vec = f32 ? 4 : 2;
    for (int i = 0; i < ns; ++i) {
        if (k[i] > GS_MAXK) return hipErrorInvalidValue;
        vec = std::min(vec, vec_of(n, ld, f32, V[i], u[i]));
    }
    const int g = blas_grid(n / vec);
    const dim3 gd(g, ns);
    if (f32) {
        UpdSys<float> a[2] = {};
        ScaleSys<float> b[2] = {};
        for (int i = 0; i < ns; ++i) {
            a[i] = UpdSys<float>{(const float*)V[i], k[i], h[i], (float*)u[i], part[i]};
            b[i] = ScaleSys<float>{(float*)u[i], part[i], nrm2[i]};
        }
        if (vec == 4)
            hipLaunchKernelGGL((gemv_sub_norm_kernel<float, 4>), gd, dim3(BLAS_THREADS), 0, st, a[0], a[1], ld, n);
        else
            hipLaunchKernelGGL((gemv_sub_norm_kernel<float, 1>), gd, dim3(BLAS_THREADS), 0, st, a[0], a[1], ld, n);
        hipLaunchKernelGGL(sum_scale_kernel<float>, dim3(blas_grid(n), ns), dim3(BLAS_THREADS), 0, st, b[0], b[1], n,
                           g);
    } else {
        UpdSys<double> a[2] = {};
        ScaleSys<double> b[2] = {};
        for (int i = 0; i < ns; ++i) {
            a[i] = UpdSys<double>{(const double*)V[i], k[i], h[i], (double*)u[i], part[i]};
            b[i] = ScaleSys<double>{(double*)u[i], part[i], nrm2[i]};
        }
        if (vec == 2)
            hipLaunchKernelGGL((gemv_sub_norm_kernel<double, 2>), gd, dim3(BLAS_THREADS), 0, st, a[0], a[1], ld, n);
        else
            hipLaunchKernelGGL((gemv_sub_norm_kernel<double, 1>), gd, dim3(BLAS_THREADS), 0, st, a[0], a[1], ld, n);
        hipLaunchKernelGGL(sum_scale_kernel<double>, dim3(blas_grid(n), ns), dim3(BLAS_THREADS), 0, st, b[0], b[1], n,
                           g);
    }
    return hipGetLastError();
}

hipError_t blas_gs_update_normalize(const void* V, size_t ld, int k, const double* h, void* u, size_t n, int f32,
                                    double* part, double* nrm2, hipStream_t st) {
    return blas_gs_update_normalize_n(1, &V, ld, &k, &h, &u, n, f32, &part, &nrm2, st);
}

// For s < ns (1 or 2) systems: h1_s[i] = V_s,i . w1_s and g_s[i] = V_s,i . w2_s for i < k_s, then the
// combined two-pass coefficients h_s = 2 h1_s - G_s h1_s with G_s's column k_s-1 set from g_s
// (G_s: device, ldg x ldg); one launch per chunk of MDOT2_CHUNK columns for all systems and one
// reduction launch.  part_s: grid * 2k_s doubles; counter_s: a device word that is 0 between launches.
hipError_t blas_gs_gram_n(int ns, const void* const* V, size_t ld, const int* k, const void* const* w1,
                          const void* const* w2, size_t n, int f32, double* const* part, double* const* h1,
                          double* const* G, int ldg, double* const* h, unsigned* const* counter, hipStream_t st) {
    int vec = f32 ? 4 : 2, kmax = 0;
    for (int i = 0; i < ns; ++i) {
        if (k[i] > GS_MAXK || k[i] > ldg) return hipErrorInvalidValue;
        vec = std::min(vec, std::min(vec_of(n, ld, f32, V[i], w1[i]), vec_of(n, ld, f32, V[i], w2[i])));
        kmax = std::max(kmax, k[i]);
    }
    const int gr = blas_grid(n / vec, MDOT_GRID);
    for (int j0 = 0; j0 < kmax; j0 += MDOT2_CHUNK) {
        const size_t es = f32 ? 4 : 8;
        auto sys = [&](int i, auto* tp) {
            using T = std::remove_pointer_t<decltype(tp)>;
            GramSys<T> q{};
            if (i < ns && j0 < k[i]) {
                q.V = (const T*)((const char*)V[i] + (size_t)j0 * ld * es);
                q.w1 = (const T*)w1[i];
                q.w2 = (const T*)w2[i];
                q.part = part[i];
                q.kc = std::min(MDOT2_CHUNK, k[i] - j0);
                q.c0 = j0;
                q.off2 = k[i];
            }
            return q;
        };
        const dim3 gd(gr, ns);
        if (f32) {
            float* tag = nullptr;
            if (vec == 4)
                hipLaunchKernelGGL((mdot2_kernel<float, 4>), gd, dim3(BLAS_THREADS), 0, st, sys(0, tag), sys(1, tag),
                                   ld, n);
            else
                hipLaunchKernelGGL((mdot2_kernel<float, 1>), gd, dim3(BLAS_THREADS), 0, st, sys(0, tag), sys(1, tag),
                                   ld, n);
        } else {
            double* tag = nullptr;
            if (vec == 2)
                hipLaunchKernelGGL((mdot2_kernel<double, 2>), gd, dim3(BLAS_THREADS), 0, st, sys(0, tag),
                                   sys(1, tag), ld, n);
            else
                hipLaunchKernelGGL((mdot2_kernel<double, 1>), gd, dim3(BLAS_THREADS), 0, st, sys(0, tag),
                                   sys(1, tag), ld, n);
        }
    }
    // h1 = part columns 0..k-1, g = columns k..2k-1 (h1 and g adjacent: g = h1 + k)
    RedSys r[2] = {};
    for (int i = 0; i < ns; ++i) r[i] = RedSys{part[i], h1[i], k[i], G[i], h[i], counter[i]};
    hipLaunchKernelGGL(reduce_gram_kernel, dim3(2 * kmax, ns), dim3(BLAS_THREADS), 0, st, r[0], r[1], gr, ldg);
    return hipGetLastError();
}

hipError_t blas_gs_gram(const void* V, size_t ld, int k, const void* w1, const void* w2, size_t n, int f32,
                        double* part, double* h1, double* g, double* G, int ldg, double* h, unsigned* counter,
                        hipStream_t st) {
    if (g != h1 + k) return hipErrorInvalidValue;
    return blas_gs_gram_n(1, &V, ld, &k, &w1, &w2, n, f32, &part, &h1, &G, ldg, &h, &counter, st);
}

// type codes: 0 = double, 1 = float
hipError_t blas_axpby(double a, const void* x, int tx, double b, void* y, int ty, size_t n, hipStream_t st) {
    int g = blas_grid(n);
    if (tx == 0 && ty == 0)
        hipLaunchKernelGGL((axpby_kernel<double, double>), dim3(g), dim3(BLAS_THREADS), 0, st, a, (const double*)x, b,
                           (double*)y, n);
    else if (tx == 0 && ty == 1)
        hipLaunchKernelGGL((axpby_kernel<double, float>), dim3(g), dim3(BLAS_THREADS), 0, st, a, (const double*)x, b,
                           (float*)y, n);
    else if (tx == 1 && ty == 0)
        hipLaunchKernelGGL((axpby_kernel<float, double>), dim3(g), dim3(BLAS_THREADS), 0, st, a, (const float*)x, b,
                           (double*)y, n);
    else
        hipLaunchKernelGGL((axpby_kernel<float, float>), dim3(g), dim3(BLAS_THREADS), 0, st, a, (const float*)x, b,
                           (float*)y, n);
    return hipGetLastError();
}

hipError_t blas_lincomb2(double a, const double* x, double b, const double* z, double* y, size_t n, hipStream_t st) {
    hipLaunchKernelGGL(lincomb2_kernel<double>, dim3(blas_grid(n)), dim3(BLAS_THREADS), 0, st, a, x, b, z, y, n);
    return hipGetLastError();
}

// y += sum_j c[j] Z_j (Z of type tz, y of type ty)
hipError_t blas_gemv_add(const void* Z, int tz, size_t ld, int k, const double* c, void* y, int ty, size_t n,
                         hipStream_t st) {
    int g = blas_grid(n);
    for (int j0 = 0; j0 < k; j0 += 8) {
        Coef8 cc;
        int kc = k - j0 < 8 ? k - j0 : 8;
        for (int j = 0; j < 8; ++j) cc.c[j] = j < kc ? c[j0 + j] : 0.0;
        if (tz == 0 && ty == 0)
            hipLaunchKernelGGL((gemv_add_kernel<double, double>), dim3(g), dim3(BLAS_THREADS), 0, st,
                               (const double*)Z + j0 * ld, ld, kc, cc, (double*)y, n);
        else if (tz == 1 && ty == 1)
            hipLaunchKernelGGL((gemv_add_kernel<float, float>), dim3(g), dim3(BLAS_THREADS), 0, st,
                               (const float*)Z + j0 * ld, ld, kc, cc, (float*)y, n);
        else if (tz == 1 && ty == 0)
            hipLaunchKernelGGL((gemv_add_kernel<float, double>), dim3(g), dim3(BLAS_THREADS), 0, st,
                               (const float*)Z + j0 * ld, ld, kc, cc, (double*)y, n);
        else
            hipLaunchKernelGGL((gemv_add_kernel<double, float>), dim3(g), dim3(BLAS_THREADS), 0, st,
                               (const double*)Z + j0 * ld, ld, kc, cc, (float*)y, n);
    }
    return hipGetLastError();
}

hipError_t blas_nonfinite(const void* x, int f32, size_t n, int* status, hipStream_t st) {
    int g = blas_grid(n);
    if (f32)
        hipLaunchKernelGGL(nonfinite_kernel<float>, dim3(g), dim3(BLAS_THREADS), 0, st, (const float*)x, n, status);
    else
        hipLaunchKernelGGL(nonfinite_kernel<double>, dim3(g), dim3(BLAS_THREADS), 0, st, (const double*)x, n, status);
    return hipGetLastError();
}
