// Internal declarations of libhbpc (not part of the public ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <cstddef>
#include <string>
#include <vector>
#include "../../include/hbpc.h"
#include "dg_launch.hpp"

// ---- kernel launchers (one translation unit per family)
hipError_t dg_launch_euler(const GeomHost& g, const LaunchReq& r, int f32);
hipError_t dg_launch_advection(const GeomHost& g, const LaunchReq& r, int f32);
hipError_t dg_launch_burgers(const GeomHost& g, const LaunchReq& r, int f32);
hipError_t dg_launch_ns(const GeomHost& g, const LaunchReq& r, int f32);
hipError_t bj_invert(double* KT, const double* HT, void* SinvT, int type, int NE, int nE, double a1dt, double bc, int* status,
                     hipStream_t st);
hipError_t bj_apply(const void* SinvT, int m_type, const void* xa, const void* xc, void* yw, void* ys, int v_f32,
                    int NE, int nE, hipStream_t st);
hipError_t bj_apply_n(const void* SinvT, int m_type, const void* const* xs, void* const* ys, int nr, int v_f32,
                      int NE, int nE, hipStream_t st);
int blas_mdot_grid(size_t n);
hipError_t blas_mdot(const void* V, size_t ld, int k, const void* w, size_t n, int f32, double* part, double* h,
                     hipStream_t st);
hipError_t blas_gs_update_normalize_n(int ns, const void* const* V, size_t ld, const int* k, const double* const* h,
                                      void* const* u, size_t n, int f32, double* const* part,
                                      double* const* nrm2, hipStream_t st);
hipError_t blas_gs_gram_n(int ns, const void* const* V, size_t ld, const int* k, const void* const* w1,
                          const void* const* w2, size_t n, int f32, double* const* part, double* const* h1,
                          double* const* G, int ldg, double* const* h, unsigned* const* counter, hipStream_t st);
hipError_t blas_gs_update_normalize(const void* V, size_t ld, int k, const double* h, void* u, size_t n, int f32,
                                    double* part, double* nrm2, hipStream_t st);
hipError_t blas_gs_gram(const void* V, size_t ld, int k, const void* w1, const void* w2, size_t n, int f32,
                        double* part, double* h1, double* g, double* G, int ldg, double* h, unsigned* counter,
                        hipStream_t st);
hipError_t blas_axpby(double a, const void* x, int tx, double b, void* y, int ty, size_t n, hipStream_t st);
hipError_t blas_lincomb2(double a, const double* x, double b, const double* z, double* y, size_t n, hipStream_t st);
hipError_t blas_gemv_add(const void* Z, int tz, size_t ld, int k, const double* c, void* y, int ty, size_t n,
                         hipStream_t st);
hipError_t blas_nonfinite(const void* x, int f32, size_t n, int* status, hipStream_t st);
hipError_t mlp_gemm(const float* A, long long a_r, long long a_c, const float* B, const uint16_t* B16, long long b_r,
                    long long b_c, float* C, long long ldc, const float* bias, const float* mask, long long ldm,
                    int mask_mul, int M, int N, int K, int relu, int accumulate, int bf16, float* ws,
                    size_t ws_floats, hipStream_t st);
hipError_t mlp_to_bf16(const float* x, uint16_t* y, long long n, hipStream_t st);
hipError_t mlp_ew_mul(const float* a, const float* b, float* out, long long n, hipStream_t st);
hipError_t mlp_ew_split(const float* dh, const float* g, const float* a, float* da, float* dz, long long n,
                        int relu_mask, hipStream_t st);
hipError_t mlp_ew_relu_mask(float* x, const float* g, long long n, hipStream_t st);
hipError_t mlp_colsum(const float* X, long long ld, int M, int N, float* out, hipStream_t st);
hipError_t mlp_mse_grad(const float* Y, const float* T, float* dY, long long n, float scale, double* part, int nblk,
                        hipStream_t st);
hipError_t mlp_adam(float* th, uint16_t* th16, const float* g, float* m, float* v, long long n, float lr, float b1,
                    float b2, float eps, int t, hipStream_t st);
hipError_t mlp_features(const void* rt, const void* w, const void* dw, int f32, const int* elems, int nb, int D,
                        const int* nel, int ne, float a1dt, float bc, float* X, float* tgt, float* scale, int part,
                        hipStream_t st);
hipError_t mlp_rescale(const float* Y, const float* scale, void* out, int f32, long long n, int ne, hipStream_t st);
hipError_t mlp_gather(const float* src, long long ld, const int* idx, int rows, int cols, float* dst, hipStream_t st);
hipError_t mlp_sum_parts(const double* part, int n, double* acc, hipStream_t st);
hipError_t mlp_randn(void* out, int f32, long long n, unsigned long long seed, hipStream_t st);
hipError_t mlp_uniform(float* out, long long n, float lim, unsigned long long seed, hipStream_t st);

// ---- 1-D operators (host, FP64)
struct Basis1DHost {
    int N, NP;
    std::vector<double> xi, w, Dhat /*NP*NP, Dhat[i*NP+lam]*/, lp, lm, lhp, lhm;
    std::vector<double> Dstr /*NP*NP, Dstr[i*NP+lam] = l_lam'(xi_i)*/, lDp, lDm;
    double cp = 0.0, cm = 0.0;
};
bool basis1d_build(int N, int kind, Basis1DHost& out);
std::vector<double> basis_table(const Basis1DHost& b);

typedef hipError_t (*FamilyLauncher)(const GeomHost&, const LaunchReq&, int);

// mesh / degree / equation / flux checks and the kernels' geometry (basis pointers left null);
// returns HBPC_OK or an error code with its message
int geom_configure(const hbpc_mesh* mesh, int N, int equation, const hbpc_params* prm, Basis1DHost& basis,
                   GeomHost& g, FamilyLauncher& launch, int& visc, int& ns, std::string& msg);

// ---- error carrier
struct HbpcError {
    int code;
    std::string msg;
};

struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
};

constexpr int KC_MAXCLS = 24;

// Buffers of one stage system of the paired corrector solves (HBPC_PC_PAIRED): the first system
// uses the context's own buffers, the second these (allocated on first use).
struct StageSys {
    double *X, *G, *dX, *rhs, *b, *trw, *trs;
    float *X32, *trw32, *trs32;
    char *V, *Z;
    void* kv;                 // PCPRE products a | c (type of the Krylov vectors)
    double *part, *dres, *dgram, *hres;
    unsigned* dcount;
    int lpc;                  // learned preconditioner active for this system's solve
    float *G1, *G2;           // its network gates at the current linearisation state
    double* trd1;             // traces of a JVP input (2 tsz values: dw then dsigma), FP64 / FP32
    float* trd1_32;
};

struct hbpc_ctx {
    hbpc_mesh mesh;
    hbpc_params prm;
    int N, NP, D, NV, NN, NFP, NE, nE, equation;
    size_t ndof, n2, tsz;     // tsz: trace values per field
    GeomHost geom;
    Basis1DHost basis;
    FamilyLauncher launch;
    hipStream_t stream;
    std::string err;

    // FP64 state
    double* W[4];             // stage values
    double* R1all;            // s x ndof
    double* R2all;            // s x ndof
    double* Wn[4];            // corrector targets
    double* X;                // Newton iterate (w | sigma), 2 ndof
    double* b;
    double* G;                // 2 ndof
    double* dX;               // 2 ndof, FP64 accumulation of the Krylov solution
    double* rhs;              // 2 ndof
    double* tmp[4];           // ndof scratch
    double* trw; double* trs; double* trd1; double* trd2;   // FP64 traces
    double* basis64; float* basis32;                         // 1-D operators on the device
    int visc;                                                // BR1 viscous terms (Burgers)
    int ns;                                                  // BR2 viscous terms (Navier-Stokes)
    void* nsg[2][4];          // BR2: each element's viscous flux at its face points per jet component, [FP64|FP32][component]
    void* qtr[2][4];                                         // BR1 lifted-gradient traces [f32][field]
    // FP32 snapshots
    float* X32;               // 2 ndof
    float* trw32; float* trs32; float* trd1_32; float* trd2_32;
    // Krylov (type chosen by precision): V (m+1) x n2, Z m x n2, u n2
    void* V; void* Z; void* kv;        // kv: 3 x n2 work (pc pre-products a|c, residual)
    int kr_f32;                        // type of V/Z
    int m_alloc;
    // BJ_ext
    double* KT;               // chunk_e x NE x NE (column-major blocks)
    double* HT;               // BJ^H_ext: Hessian blocks, same layout (allocated on first use)
    void* Sinv;               // nE x NE x NE: the active slot's blocks
    int sinv_f32;             // S^-1 feeds FP32 vectors (stored FP32 or FP16)
    int sinv_type;            // storage: 0 FP64, 1 FP32, 2 FP16
    size_t kt_chunk;          // elements per K build chunk (<= 4 GiB of FP64 blocks)
    double pc_a1dt, pc_bc;
    int pc_valid;
    int pc_hess;              // the active blocks are BJ^H_ext's (apply: y, vs + K y)
    // S^-1 slots: 0 for the predictor (and every solve unless blocks are kept per stage), l - 1
    // for corrector stage l when they are
    void* Sinv_slot[4];
    int sinv_type_slot[4], slot_valid[4], slot_hess[4];
    double slot_a1dt[4], slot_bc[4];
    int cur_slot;
    int pc_kept;              // the active slot's blocks serve the current stage solve as they are
    int pc_steps;             // HBPC_PC_ACROSS_STEPS: steps since the kept blocks were invalidated
    // reductions
    double* part;             // blas partials
    double* dres;             // device results: one Arnoldi slot (arn_len), then 64 words (norm, loss)
    size_t arn_len;           // 3 (m + 1) + 8: h1 | g, ||u||^2, h of one Arnoldi iteration
    double* dgram;            // Gram matrix V^T V of the current FGMRES cycle, (m+1) x (m+1)
    unsigned* dcount;         // grid-wide hand-over counters of the fused reductions (0 between launches)
    double* hres;             // pinned host copies: two Arnoldi slots of arn_len, then 64 words
    hipEvent_t arn_ev[2];     // Arnoldi results of iteration j copied to slot j % 2
    StageSys pair;            // second system of HBPC_PC_PAIRED (null pointers until used)
    int* dstatus;
    // FD scratch (allocated on demand)
    double* fd[6];
    // learned preconditioner (network: n_r residual + n_w state inputs -> H -> H -> NE)
    int mlp_nin, mlp_nr, mlp_H;
    size_t mlp_np;
    float* theta; float* adam_m; float* adam_v; float* mgrad;   // FP32 parameters, moments, gradient
    uint16_t* theta16;                                          // BF16 copy of theta (matrix-core operand)
    float* gemm_ws; size_t gemm_ws_floats;                      // split-k partial sums of the network GEMMs
    int adam_t, mlp_ready;
    float* ap_X; float* ap_G1; float* ap_G2; float* ap_H1; float* ap_H2; float* ap_Y; float* ap_s;   // nE rows
    float* tr_buf; int tr_rows;                                        // training buffers (batch rows)
    int lpc_active;            // learned PC in use for the current stage solve
    int lpc_snap;              // hbpc_pc_build in learned mode: -1 none, 0 FP64, 1 FP32 snapshot
    int* tr_idx_dev; size_t tr_idx_cap;
    float* col_X; float* col_T; size_t col_cap, col_count; int col_per, col_source, col_every;
    unsigned long long col_seed, col_draws;
    int* col_elems;
    // statistics of the last step
    hbpc_stats st;
    int cur_solve;
    int verbose;              // HBPC_VERBOSE=1: Newton progress on stderr
    // kernel timing
    int prof;
    int prof_only;            // >= 0: record only this kernel class
    std::vector<hipEvent_t> ev;          // pairs (start, stop)
    std::vector<int> ev_class;
    std::vector<double> ev_bytes, ev_flops;
    size_t ev_used;
    int kp_launch[KC_MAXCLS];
    double kp_ms[KC_MAXCLS], kp_bytes[KC_MAXCLS], kp_flops[KC_MAXCLS];
};

enum { KC_TRACE = 0, KC_R1, KC_R2, KC_RES, KC_JVP, KC_KCOL, KC_PCPRE, KC_BJAPPLY, KC_BJINV, KC_MDOT, KC_GEMV,
       KC_VEC, KC_GSDOT, KC_GSUPD, KC_LIN, KC_FEAT, KC_GEMM, KC_MLPV, KC_NSGRAD, KC_BJAPPLY4, KC_COUNT };

// helpers implemented in ops.cpp
int op_launch(hbpc_ctx* c, const LaunchReq& r, int f32);
LaunchReq op_req(hbpc_ctx* c, int op);
