// Kernels of the learned per-element preconditioner: feature gather, dense
// layers (BF16 matrix cores with FP32 accumulation, or plain FP32), loss,
// backward helpers and Adam.
//
// GEMM: C[M x N] = A[M x K] B[K x N] with general strides for A and B (so
// transposed operands need no copies), FP32 activations, optional bias, ReLU
// and a mask (C *= (mask > 0), or C *= mask for gating), FP32 output.
//
// BF16 mode (gfx950 matrix cores): block tile 64 x 64 x 32, 256 threads, each
// wave a 32 x 32 quarter as 2 x 2 tiles of v_mfma_f32_16x16x32_bf16 (one MFMA
// per 16 x 16 tile and 32-deep k step).  FP32 operands are rounded to BF16
// (round to nearest even) as they are written to LDS; a weight operand comes
// from the BF16 copy of the parameters kept beside the FP32 master copy, so
// it is read as BF16 from HBM.  Each thread stages 8 consecutive values of the
// operand's unit-stride dimension (vector loads where aligned); the next k
// tile is loaded into registers while the matrix cores work on the current
// one.  Small products with a long k (the weight gradients of a mini-batch)
// are split over k into a work space and summed in a fixed order, so results
// do not depend on scheduling.
//
// FP32 mode: the same 64 x 64 x 32 tiling with FP32 FMAs, 4 x 4 outputs per thread.
#include <hip/hip_runtime.h>
#include <algorithm>
#include <cstdint>

namespace {

constexpr int BM = 64, BN = 64, BK = 32;
constexpr int KP = BK + 8;   // BF16 LDS row pitch: 80 bytes, rows 16-byte aligned

__device__ __forceinline__ uint16_t f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);   // round to nearest even (finite inputs)
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ uint32_t pack2(float lo, float hi) {
    return (uint32_t)f2bf(lo) | ((uint32_t)f2bf(hi) << 16);
}

struct GemmArgs {
    const float* A; long long a_r, a_c;   // A(i,k) = A[i*a_r + k*a_c]
    const float* B; long long b_r, b_c;   // B(k,j) = B[k*b_r + j*b_c]
    const uint16_t* B16;                  // BF16 copy of B with the same strides (null: round B)
    float* C; long long ldc;              // C(i,j) = C[i*ldc + j]
    const float* bias;                    // bias[j] or null
    const float* mask; long long ldm;     // mask(i,j) (null: none)
    int mask_mul;                         // 0: multiply by (mask > 0), 1: multiply by mask
    int M, N, K;
    int relu;
    int accumulate;                       // C += result
    float* ws;                            // split-k partial sums [split][M][N] (null: no split)
    int kchunk;                           // k range of one split (multiple of BK)
    int vec_a, vec_b;                     // 1: the staged 8-runs of A / B may use 16-byte loads, 2: 8-byte
};

typedef float float4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));

__device__ __forceinline__ void gemm_store(const GemmArgs& g, int i, int j, float v) {
    if (i >= g.M || j >= g.N) return;
    if (g.bias) v += g.bias[j];
    if (g.relu) v = v > 0.f ? v : 0.f;
    if (g.mask) {
        const float mk = g.mask[(long long)i * g.ldm + j];
        v = g.mask_mul ? v * mk : (mk > 0.f ? v : 0.f);
    }
    float* c = g.C + (long long)i * g.ldc + j;
    *c = g.accumulate ? *c + v : v;
}

// Eight FP32 values p[0], p[s], ..., p[7s], the first n of them in range (the rest 0).
// vec: 1 = p 16-byte aligned and s == 1, 2 = 8-byte aligned and s == 1.
__device__ __forceinline__ void load8(const float* __restrict__ p, long long s, int n, int vec, float v[8]) {
    if (n >= 8 && vec == 1) {
        const float4 x = *(const float4*)p, y = *(const float4*)(p + 4);
        v[0] = x.x; v[1] = x.y; v[2] = x.z; v[3] = x.w; v[4] = y.x; v[5] = y.y; v[6] = y.z; v[7] = y.w;
    } else if (n >= 8 && vec == 2) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const float2 x = *(const float2*)(p + 2 * q);
            v[2 * q] = x.x;
            v[2 * q + 1] = x.y;
        }
    } else {
#pragma unroll
        for (int q = 0; q < 8; ++q) v[q] = q < n ? p[q * s] : 0.f;
    }
}

// The same for a BF16 source (vec 1: 16-byte aligned, s == 1).
__device__ __forceinline__ uint4 load8_bf(const uint16_t* __restrict__ p, long long s, int n, int vec) {
    if (n >= 8 && vec == 1) return *(const uint4*)p;
    uint16_t h[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) h[q] = q < n ? p[q * s] : (uint16_t)0;
    return make_uint4(h[0] | ((uint32_t)h[1] << 16), h[2] | ((uint32_t)h[3] << 16), h[4] | ((uint32_t)h[5] << 16),
                      h[6] | ((uint32_t)h[7] << 16));
}

// One operand tile in LDS as T[r][k] (r = row of A or column of B, k contiguous), staged
// from a matrix X(r, k) = X[r*s_r + k*s_c] with r in [r0, r0 + 64) (limit R) and
// k in [k0, k0 + 32) (limit k1).  If s_r == 1 (r is the unit-stride dimension) each
// thread holds 8 consecutive r of one k, else 8 consecutive k of one r.
struct Stage {
    float v[8];
    uint4 h;
    int rr, kk;      // tile coordinates of the thread's run
    bool along_r;
};

__device__ __forceinline__ void stage_setup(Stage& st, bool along_r, int tid) {
    st.along_r = along_r;
    if (along_r) {
        st.kk = tid >> 3;
        st.rr = (tid & 7) * 8;
    } else {
        st.rr = tid >> 2;
        st.kk = (tid & 3) * 8;
    }
}

__device__ __forceinline__ void stage_load(Stage& st, const float* X, const uint16_t* X16, long long s_r,
                                           long long s_c, int r0, int R, int k0, int k1, int vec) {
    const int gr = r0 + st.rr, gk = k0 + st.kk;
    int n;
    long long off, step;
    if (st.along_r) {
        n = gk < k1 ? min(8, R - gr) : 0;
        off = (long long)gr * s_r + (long long)gk * s_c;
        step = s_r;
    } else {
        n = gr < R ? min(8, k1 - gk) : 0;
        off = (long long)gr * s_r + (long long)gk * s_c;
        step = s_c;
    }
    if (n < 0) n = 0;
    if (X16) st.h = load8_bf(X16 + (n > 0 ? off : 0), step, n, vec);
    else load8(X + (n > 0 ? off : 0), step, n, vec, st.v);
}

__device__ __forceinline__ void stage_store(const Stage& st, uint16_t (*T)[KP], bool bf_src) {
    uint4 h = st.h;
    if (!bf_src)
        h = make_uint4(pack2(st.v[0], st.v[1]), pack2(st.v[2], st.v[3]), pack2(st.v[4], st.v[5]),
                       pack2(st.v[6], st.v[7]));
    if (st.along_r) {
        const uint32_t w[4] = {h.x, h.y, h.z, h.w};
#pragma unroll
        for (int q = 0; q < 8; ++q) T[st.rr + q][st.kk] = (uint16_t)(w[q >> 1] >> (16 * (q & 1)));
    } else {
        *(uint4*)&T[st.rr][st.kk] = h;
    }
}

__global__ void __launch_bounds__(256) gemm_mfma_kernel(GemmArgs g) {
    __shared__ __align__(16) uint16_t As[BM][KP];
    __shared__ __align__(16) uint16_t Bs[BN][KP];
    const int tid = threadIdx.x;
    const int i0 = blockIdx.y * BM, j0 = blockIdx.x * BN;
    const int wave = tid >> 6, lane = tid & 63;
    const int wi = (wave >> 1) * 32, wj = (wave & 1) * 32;   // wave quarter of the block tile
    const int kb = blockIdx.z * g.kchunk, ke = min(g.K, kb + g.kchunk);

    // A(i, k): r = i; B(k, j) as T(r = j, k)
    Stage sa, sb;
    stage_setup(sa, g.a_r == 1 && g.a_c != 1, tid);
    stage_setup(sb, g.b_c == 1 && g.b_r != 1, tid);
    float4_t acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = (float4_t){0.f, 0.f, 0.f, 0.f};

    // v_mfma_f32_16x16x32_bf16: lane l supplies A[l%16][8(l/16)..+7] and B[8(l/16)..+7][l%16];
    // it receives D[4(l/16)+r][l%16], r = 0..3
    const int lr = lane & 15, lk = (lane >> 4) * 8;
    if (kb < ke) {
        stage_load(sa, g.A, nullptr, g.a_r, g.a_c, i0, g.M, kb, ke, g.vec_a);
        stage_load(sb, g.B, g.B16, g.b_c, g.b_r, j0, g.N, kb, ke, g.vec_b);
    }
    for (int k0 = kb; k0 < ke; k0 += BK) {
        stage_store(sa, As, false);
        stage_store(sb, Bs, g.B16 != nullptr);
        __syncthreads();
        if (k0 + BK < ke) {   // next tile in flight while this one is multiplied
            stage_load(sa, g.A, nullptr, g.a_r, g.a_c, i0, g.M, k0 + BK, ke, g.vec_a);
            stage_load(sb, g.B, g.B16, g.b_c, g.b_r, j0, g.N, k0 + BK, ke, g.vec_b);
        }
        bf16x8_t af[2], bfr[2];
#pragma unroll
        for (int a = 0; a < 2; ++a) af[a] = *(const bf16x8_t*)&As[wi + 16 * a + lr][lk];
#pragma unroll
        for (int b = 0; b < 2; ++b) bfr[b] = *(const bf16x8_t*)&Bs[wj + 16 * b + lr][lk];
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
                acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[a], bfr[b], acc[a][b], 0, 0, 0);
        __syncthreads();
    }
    const int lq = (lane >> 4) * 4;
    if (g.ws) {   // split-k partial sums, epilogue in gemm_split_sum_kernel
        float* P = g.ws + (size_t)blockIdx.z * g.M * g.N;
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int i = i0 + wi + 16 * a + lq + r, j = j0 + wj + 16 * b + lr;
                    if (i < g.M && j < g.N) P[(size_t)i * g.N + j] = acc[a][b][r];
                }
        return;
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) gemm_store(g, i0 + wi + 16 * a + lq + r, j0 + wj + 16 * b + lr, acc[a][b][r]);
}

// C(i, j) <- epilogue(sum over the splits of ws[s][i][j], in split order)
__global__ void __launch_bounds__(256) gemm_split_sum_kernel(GemmArgs g, int splits) {
    const size_t MN = (size_t)g.M * g.N;
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < MN; t += (size_t)gridDim.x * blockDim.x) {
        float s = 0.f;
        for (int z = 0; z < splits; ++z) s += g.ws[z * MN + t];
        gemm_store(g, (int)(t / g.N), (int)(t % g.N), s);
    }
}

__global__ void __launch_bounds__(256) gemm_f32_kernel(GemmArgs g) {
    // LDS tiles: As[i][k] and Bs[j][k] (k contiguous for both)
    __shared__ float As32[BM][BK + 1];
    __shared__ float Bs32[BN][BK + 1];
    const int tid = threadIdx.x;
    const int i0 = blockIdx.y * BM, j0 = blockIdx.x * BN;
    float accf[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) accf[a][b] = 0.f;
    const int ti = tid / 16, tj = tid % 16;   // 4 x 4 outputs at (ti + 16a, tj + 16b)

    for (int k0 = 0; k0 < g.K; k0 += BK) {
        // walk each operand along its unit stride
        for (int idx = tid; idx < BM * BK; idx += 256) {
            const int ii = g.a_c == 1 ? idx / BK : idx % BM;
            const int kk = g.a_c == 1 ? idx % BK : idx / BM;
            const int gi = i0 + ii, gk = k0 + kk;
            As32[ii][kk] = (gi < g.M && gk < g.K) ? g.A[gi * g.a_r + gk * g.a_c] : 0.f;
        }
        for (int idx = tid; idx < BN * BK; idx += 256) {
            const int jj = g.b_c == 1 ? idx % BN : idx / BK;
            const int kk = g.b_c == 1 ? idx / BN : idx % BK;
            const int gj = j0 + jj, gk = k0 + kk;
            Bs32[jj][kk] = (gj < g.N && gk < g.K) ? g.B[gk * g.b_r + gj * g.b_c] : 0.f;
        }
        __syncthreads();
#pragma unroll 4
        for (int kk = 0; kk < BK; ++kk) {
            float ra[4], rb[4];
#pragma unroll
            for (int a = 0; a < 4; ++a) ra[a] = As32[ti + 16 * a][kk];
#pragma unroll
            for (int b = 0; b < 4; ++b) rb[b] = Bs32[tj + 16 * b][kk];
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b) accf[a][b] += ra[a] * rb[b];
        }
        __syncthreads();
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) gemm_store(g, i0 + ti + 16 * a, j0 + tj + 16 * b, accf[a][b]);
}

// column sums: out[j] (+)= sum_i X[i*ld + j]
__global__ void __launch_bounds__(256) colsum_kernel(const float* __restrict__ X, long long ld, int M, int N,
                                                     float* __restrict__ out) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= N) return;
    double s = 0.0;
    for (int i = 0; i < M; ++i) s += X[i * ld + j];
    out[j] = (float)s;
}

// dY = 2 (Y - T) / (M N); per-block partial of sum (Y - T)^2
__global__ void __launch_bounds__(256) mse_grad_kernel(const float* __restrict__ Y, const float* __restrict__ T,
                                                       float* __restrict__ dY, long long n, float scale,
                                                       double* __restrict__ part) {
    __shared__ double sh[4];
    double acc = 0.0;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        const float d = Y[i] - T[i];
        dY[i] = 2.f * d * scale;
        acc += (double)d * d;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0] + sh[1] + sh[2] + sh[3];
}

__global__ void __launch_bounds__(256) adam_kernel(float* __restrict__ th, uint16_t* __restrict__ th16,
                                                   const float* __restrict__ g, float* __restrict__ m,
                                                   float* __restrict__ v, long long n, float lr, float b1, float b2,
                                                   float eps, float c1, float c2) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.f - b1) * gi;
        const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        const float t = th[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
        th[i] = t;
        if (th16) th16[i] = f2bf(t);
    }
}

// y = BF16(x), round to nearest even
__global__ void __launch_bounds__(256) to_bf16_kernel(const float* __restrict__ x, uint16_t* __restrict__ y,
                                                      long long n) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        y[i] = f2bf(x[i]);
}

// Feature rows of the learned preconditioner, one block per sample:
// X[s] = [rt tiles of (e, its 2d face neighbours) / scale, w tiles of the same, c1, c2],
// scale = RMS of the rt patch (+1e-30); targets (optional) = dw_e / scale.
// part: bit 0 = residual tiles (and scale, targets), bit 1 = state tiles and coefficients
template <typename T>
__global__ void __launch_bounds__(256) features_kernel(const T* __restrict__ rt, const T* __restrict__ w,
                                                       const T* __restrict__ dw, const int* __restrict__ elems,
                                                       int nb, int D, int nel0, int nel1, int nel2, int ne,
                                                       float c1, float c2, float* __restrict__ X,
                                                       float* __restrict__ tgt, float* __restrict__ scale,
                                                       int part) {
    __shared__ int patch[7];
    __shared__ double red[4];
    const int s = blockIdx.x;
    if (s >= nb) return;
    const int e = elems ? elems[s] : s;
    const int np = 2 * D + 1;
    const int nin = 2 * np * ne + 2;
    if (e < 0 || e >= nel0 * nel1 * nel2) {   // element index out of range: zero row
        for (int i = threadIdx.x; i < nin; i += blockDim.x) X[(size_t)s * nin + i] = 0.f;
        if (threadIdx.x == 0 && scale) scale[s] = 0.f;
        if (tgt)
            for (int i = threadIdx.x; i < ne; i += blockDim.x) tgt[(size_t)s * ne + i] = 0.f;
        return;
    }
    if (threadIdx.x == 0) {
        int c[3] = {e % nel0, D > 1 ? (e / nel0) % nel1 : 0, D > 2 ? e / (nel0 * nel1) : 0};
        int n[3] = {nel0, nel1, nel2};
        patch[0] = e;
        for (int m = 0; m < D; ++m)
            for (int sd = 0; sd < 2; ++sd) {
                int cc[3] = {c[0], c[1], c[2]};
                cc[m] = (cc[m] + (sd ? 1 : -1) + n[m]) % n[m];
                patch[1 + 2 * m + sd] = cc[0] + nel0 * (cc[1] + nel1 * cc[2]);
            }
    }
    __syncthreads();
    float* row = X + (size_t)s * nin;
    if (part & 2) {
        for (int i = threadIdx.x; i < np * ne; i += blockDim.x)
            row[np * ne + i] = (float)w[(size_t)patch[i / ne] * ne + (i % ne)];
        if (threadIdx.x == 0) {
            row[nin - 2] = c1;
            row[nin - 1] = c2;
        }
    }
    if (!(part & 1)) return;
    double acc = 0.0;
    for (int i = threadIdx.x; i < np * ne; i += blockDim.x) {
        const double v = (double)rt[(size_t)patch[i / ne] * ne + (i % ne)];
        acc += v * v;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    const double sc = sqrt((red[0] + red[1] + red[2] + red[3]) / (np * ne)) + 1e-30;
    const double isc = 1.0 / sc;
    for (int i = threadIdx.x; i < np * ne; i += blockDim.x)
        row[i] = (float)((double)rt[(size_t)patch[i / ne] * ne + (i % ne)] * isc);
    if (threadIdx.x == 0 && scale) scale[s] = (float)sc;
    if (tgt)
        for (int i = threadIdx.x; i < ne; i += blockDim.x)
            tgt[(size_t)s * ne + i] = (float)((double)dw[(size_t)e * ne + i] * isc);
}

// out[e][i] = scale[e] * Y[e][i] (w block of the preconditioned vector)
template <typename T>
__global__ void __launch_bounds__(256) rescale_kernel(const float* __restrict__ Y, const float* __restrict__ scale,
                                                      T* __restrict__ out, long long n, int ne) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        out[i] = (T)((double)Y[i] * (double)scale[i / ne]);
}

// out = a * b
__global__ void __launch_bounds__(256) ew_mul_kernel(const float* __restrict__ a, const float* __restrict__ b,
                                                     float* __restrict__ out, long long n) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        out[i] = a[i] * b[i];
}

// backward through h = a * g (g = relu(z)): da = dh * g, dz = dh * a [* (g > 0)]
__global__ void __launch_bounds__(256) ew_split_kernel(const float* __restrict__ dh, const float* __restrict__ g,
                                                       const float* __restrict__ a, float* __restrict__ da,
                                                       float* __restrict__ dz, long long n, int relu_mask) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        const float d = dh[i], gi = g[i];
        da[i] = d * gi;
        const float z = d * a[i];
        dz[i] = relu_mask ? (gi > 0.f ? z : 0.f) : z;
    }
}

// x *= (g > 0)
__global__ void __launch_bounds__(256) ew_relu_mask_kernel(float* __restrict__ x, const float* __restrict__ g,
                                                           long long n) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        if (!(g[i] > 0.f)) x[i] = 0.f;
}

// splitmix64 finaliser (Steele, Lea & Flood 2014) of the counter value seed + (k + 1) * golden gamma
__device__ __forceinline__ unsigned long long sm64_at(unsigned long long seed, unsigned long long k) {
    unsigned long long z = seed + (k + 1ull) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// standard normal values by the Box-Muller transform of two counter-based uniforms in (0, 1]
template <typename T>
__global__ void __launch_bounds__(256) randn_kernel(T* __restrict__ out, long long n, unsigned long long seed) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        const double u1 = ((double)(sm64_at(seed, 2ull * i) >> 11) + 1.0) * 0x1.0p-53;
        const double u2 = (double)(sm64_at(seed, 2ull * i + 1ull) >> 11) * 0x1.0p-53;
        out[i] = (T)(sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2));
    }
}

// out[i] = lim (2u - 1), u uniform in [0, 1) from the top 24 bits of a splitmix64 counter value
__global__ void __launch_bounds__(256) uniform_kernel(float* __restrict__ out, long long n, float lim,
                                                      unsigned long long seed) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        const float u = (float)(sm64_at(seed, (unsigned long long)i) >> 40) * 0x1.0p-24f;
        out[i] = lim * (2.f * u - 1.f);
    }
}

// out[r][:] = src[idx[r]][:] (mini-batch gather)
__global__ void __launch_bounds__(256) gather_rows_kernel(const float* __restrict__ src, long long ld,
                                                          const int* __restrict__ idx, int cols,
                                                          float* __restrict__ dst) {
    const float* s = src + (size_t)idx[blockIdx.x] * ld;
    float* d = dst + (size_t)blockIdx.x * cols;
    for (int c = threadIdx.x; c < cols; c += blockDim.x) d[c] = s[c];
}

// *acc += sum of the n block partials (one thread)
__global__ void sum_parts_kernel(const double* __restrict__ part, int n, double* __restrict__ acc) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += part[i];
    *acc += s;
}

}  // namespace

// ------------------------------------------------------------------ launchers
static int vec_flag(const void* p, long long other, int esize) {
    const uintptr_t a = (uintptr_t)p;
    const int per16 = 16 / esize;   // elements of one 16-byte load
    if (a % 16 == 0 && other % per16 == 0) return 1;
    if (esize == 4 && a % 8 == 0 && other % 2 == 0) return 2;
    return 0;
}

hipError_t mlp_gemm(const float* A, long long a_r, long long a_c, const float* B, const uint16_t* B16, long long b_r,
                    long long b_c, float* C, long long ldc, const float* bias, const float* mask, long long ldm,
                    int mask_mul, int M, int N, int K, int relu, int accumulate, int bf16, float* ws,
                    size_t ws_floats, hipStream_t st) {
    if (M <= 0 || N <= 0) return hipSuccess;
    GemmArgs g{};
    g.A = A; g.a_r = a_r; g.a_c = a_c;
    g.B = B; g.b_r = b_r; g.b_c = b_c;
    g.B16 = bf16 ? B16 : nullptr;
    g.C = C; g.ldc = ldc; g.bias = bias; g.mask = mask; g.ldm = ldm; g.mask_mul = mask_mul;
    g.M = M; g.N = N; g.K = K; g.relu = relu; g.accumulate = accumulate;
    const unsigned gx = (N + BN - 1) / BN, gy = (M + BM - 1) / BM;
    if (!bf16) {
        hipLaunchKernelGGL(gemm_f32_kernel, dim3(gx, gy), dim3(256), 0, st, g);
        return hipGetLastError();
    }
    // the unit-stride dimension of each staged 8-run (see stage_setup) and its alignment
    const bool a_along_r = a_r == 1 && a_c != 1, b_along_r = b_c == 1 && b_r != 1;
    if (a_along_r ? a_r == 1 : a_c == 1) g.vec_a = vec_flag(A, a_along_r ? a_c : a_r, 4);
    const void* bsrc = g.B16 ? (const void*)g.B16 : (const void*)B;
    if (b_along_r ? b_c == 1 : b_r == 1) g.vec_b = vec_flag(bsrc, b_along_r ? b_r : b_c, g.B16 ? 2 : 4);
    // split k when the output tiles alone cannot fill the chip
    const long long tiles = (long long)gx * gy;
    const int ksteps = (K + BK - 1) / BK;
    int splits = 1;
    if (ws && tiles < 256 && ksteps >= 8) {
        splits = (int)std::min<long long>((512 + tiles - 1) / tiles, ksteps / 4);
        splits = std::min(splits, 32);
        while (splits > 1 && (size_t)splits * M * N > ws_floats) --splits;
    }
    const int chunk = ((ksteps + splits - 1) / splits) * BK;
    splits = K > 0 ? (K + chunk - 1) / chunk : 1;
    g.kchunk = K > 0 ? chunk : BK;
    if (splits > 1) {
        g.ws = ws;
        hipLaunchKernelGGL(gemm_mfma_kernel, dim3(gx, gy, splits), dim3(256), 0, st, g);
        const size_t mn = (size_t)M * N;
        const unsigned blocks = (unsigned)std::min<size_t>(2048, (mn + 255) / 256);
        hipLaunchKernelGGL(gemm_split_sum_kernel, dim3(blocks), dim3(256), 0, st, g, splits);
    } else {
        hipLaunchKernelGGL(gemm_mfma_kernel, dim3(gx, gy, 1), dim3(256), 0, st, g);
    }
    return hipGetLastError();
}

hipError_t mlp_to_bf16(const float* x, uint16_t* y, long long n, hipStream_t st) {
    long long blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) return hipSuccess;
    hipLaunchKernelGGL(to_bf16_kernel, dim3((unsigned)blocks), dim3(256), 0, st, x, y, n);
    return hipGetLastError();
}

hipError_t mlp_colsum(const float* X, long long ld, int M, int N, float* out, hipStream_t st) {
    hipLaunchKernelGGL(colsum_kernel, dim3((N + 255) / 256), dim3(256), 0, st, X, ld, M, N, out);
    return hipGetLastError();
}

hipError_t mlp_mse_grad(const float* Y, const float* T, float* dY, long long n, float scale, double* part, int nblk,
                        hipStream_t st) {
    hipLaunchKernelGGL(mse_grad_kernel, dim3(nblk), dim3(256), 0, st, Y, T, dY, n, scale, part);
    return hipGetLastError();
}

hipError_t mlp_adam(float* th, uint16_t* th16, const float* g, float* m, float* v, long long n, float lr, float b1,
                    float b2, float eps, int t, hipStream_t st) {
    const float c1 = (float)(1.0 - pow((double)b1, t)), c2 = (float)(1.0 - pow((double)b2, t));
    long long blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(adam_kernel, dim3((unsigned)blocks), dim3(256), 0, st, th, th16, g, m, v, n, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

hipError_t mlp_features(const void* rt, const void* w, const void* dw, int f32, const int* elems, int nb, int D,
                        const int* nel, int ne, float a1dt, float bc, float* X, float* tgt, float* scale, int part,
                        hipStream_t st) {
    if (nb <= 0) return hipSuccess;
    if (f32)
        hipLaunchKernelGGL(features_kernel<float>, dim3(nb), dim3(256), 0, st, (const float*)rt, (const float*)w,
                           (const float*)dw, elems, nb, D, nel[0], nel[1], nel[2], ne, a1dt, bc, X, tgt, scale, part);
    else
        hipLaunchKernelGGL(features_kernel<double>, dim3(nb), dim3(256), 0, st, (const double*)rt, (const double*)w,
                           (const double*)dw, elems, nb, D, nel[0], nel[1], nel[2], ne, a1dt, bc, X, tgt, scale,
                           part);
    return hipGetLastError();
}

static unsigned ew_blocks(long long n) {
    long long b = (n + 255) / 256;
    return (unsigned)(b > 4096 ? 4096 : (b < 1 ? 1 : b));
}

hipError_t mlp_ew_mul(const float* a, const float* b, float* out, long long n, hipStream_t st) {
    hipLaunchKernelGGL(ew_mul_kernel, dim3(ew_blocks(n)), dim3(256), 0, st, a, b, out, n);
    return hipGetLastError();
}

hipError_t mlp_ew_split(const float* dh, const float* g, const float* a, float* da, float* dz, long long n,
                        int relu_mask, hipStream_t st) {
    hipLaunchKernelGGL(ew_split_kernel, dim3(ew_blocks(n)), dim3(256), 0, st, dh, g, a, da, dz, n, relu_mask);
    return hipGetLastError();
}

hipError_t mlp_ew_relu_mask(float* x, const float* g, long long n, hipStream_t st) {
    hipLaunchKernelGGL(ew_relu_mask_kernel, dim3(ew_blocks(n)), dim3(256), 0, st, x, g, n);
    return hipGetLastError();
}

hipError_t mlp_rescale(const float* Y, const float* scale, void* out, int f32, long long n, int ne, hipStream_t st) {
    long long blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    if (f32)
        hipLaunchKernelGGL(rescale_kernel<float>, dim3((unsigned)blocks), dim3(256), 0, st, Y, scale, (float*)out, n, ne);
    else
        hipLaunchKernelGGL(rescale_kernel<double>, dim3((unsigned)blocks), dim3(256), 0, st, Y, scale, (double*)out, n,
                           ne);
    return hipGetLastError();
}

hipError_t mlp_gather(const float* src, long long ld, const int* idx, int rows, int cols, float* dst, hipStream_t st) {
    if (rows <= 0) return hipSuccess;
    hipLaunchKernelGGL(gather_rows_kernel, dim3(rows), dim3(256), 0, st, src, ld, idx, cols, dst);
    return hipGetLastError();
}

hipError_t mlp_sum_parts(const double* part, int n, double* acc, hipStream_t st) {
    hipLaunchKernelGGL(sum_parts_kernel, dim3(1), dim3(64), 0, st, part, n, acc);
    return hipGetLastError();
}

hipError_t mlp_randn(void* out, int f32, long long n, unsigned long long seed, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    if (f32) hipLaunchKernelGGL(randn_kernel<float>, dim3(ew_blocks(n)), dim3(256), 0, st, (float*)out, n, seed);
    else hipLaunchKernelGGL(randn_kernel<double>, dim3(ew_blocks(n)), dim3(256), 0, st, (double*)out, n, seed);
    return hipGetLastError();
}

hipError_t mlp_uniform(float* out, long long n, float lim, unsigned long long seed, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(uniform_kernel, dim3(ew_blocks(n)), dim3(256), 0, st, out, n, lim, seed);
    return hipGetLastError();
}
