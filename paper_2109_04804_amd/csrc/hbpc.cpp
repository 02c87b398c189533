// libhbpc host side: context, operator wrappers, Newton-Krylov stage solver and
// the HBPC(q, k_max) driver (Algorithm 1), behind the C ABI of include/hbpc.h.
//
// Stage solve (Sec. 3.2): Newton on the extended residual
//   G(X) = (w - a1dt R1(w) + bcoef R2(w, sigma) - b,  sigma - R1(w)),
// each correction from right-preconditioned restarted FGMRES on the extended
// Jacobian (Eq. nonlinear_eqsys).  Stopping rules: Newton stops when
// ||G(X^r)|| <= eps_N ||G(X^0)|| or ||dw^r||_2 / sqrt(ndof) <= atol_dw; no iteration when
// ||G(X^0)|| <= 1e-14 sqrt(2 ndof); FGMRES starts from 0 and stops when
// ||r_j|| <= eps_G ||r_0||.  Norms are Euclidean over all coefficients.
// Initial guess X^0 = (guess, R1(guess)).
//
// Mixed precision: G, the stage vectors and X += dX stay FP64; the Krylov
// vectors, the JVP (on FP32 copies of w, sigma taken once per Newton
// iteration) and S^-1 of BJ_ext are FP32.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <rocprofiler-sdk-roctx/roctx.h>
#include "hbpc_internal.hpp"

// ------------------------------------------------------------------ tableaux (appendix)
struct Tab {
    int s;
    double c[4];
    double B1[4][4];
    double B2[4][4];
};

static bool tableau(int q, Tab& t) {
    std::memset(&t, 0, sizeof(t));
    if (q == 4) {
        t.s = 2;
        t.c[0] = 0; t.c[1] = 1;
        t.B1[1][0] = 0.5; t.B1[1][1] = 0.5;
        t.B2[1][0] = 1.0 / 12; t.B2[1][1] = -1.0 / 12;
        return true;
    }
    if (q == 6) {
        t.s = 3;
        t.c[0] = 0; t.c[1] = 0.5; t.c[2] = 1;
        t.B1[1][0] = 101.0 / 480; t.B1[1][1] = 8.0 / 30; t.B1[1][2] = 55.0 / 2400;
        t.B1[2][0] = 7.0 / 30; t.B1[2][1] = 16.0 / 30; t.B1[2][2] = 7.0 / 30;
        t.B2[1][0] = 65.0 / 4800; t.B2[1][1] = -25.0 / 600; t.B2[1][2] = -25.0 / 8000;
        t.B2[2][0] = 5.0 / 300; t.B2[2][1] = 0.0; t.B2[2][2] = -5.0 / 300;
        return true;
    }
    if (q == 8) {
        t.s = 4;
        t.c[0] = 0; t.c[1] = 1.0 / 3; t.c[2] = 2.0 / 3; t.c[3] = 1;
        const double b1[3][4] = {{6893.0 / 54432, 313.0 / 2016, 89.0 / 2016, 397.0 / 54432},
                                 {223.0 / 1701, 20.0 / 63, 13.0 / 63, 20.0 / 1701},
                                 {31.0 / 224, 81.0 / 224, 81.0 / 224, 31.0 / 224}};
        const double b2[3][4] = {{1283.0 / 272160, -851.0 / 30240, -269.0 / 30240, -163.0 / 272160},
                                 {43.0 / 8505, -16.0 / 945, -19.0 / 945, -8.0 / 8505},
                                 {19.0 / 3360, -9.0 / 1120, 9.0 / 1120, -19.0 / 3360}};
        for (int l = 1; l < 4; ++l)
            for (int j = 0; j < 4; ++j) {
                t.B1[l][j] = b1[l - 1][j];
                t.B2[l][j] = b2[l - 1][j];
            }
        return true;
    }
    return false;
}

// ------------------------------------------------------------------ error handling
namespace {
struct Fail {
    int code;
};

void set_err(hbpc_ctx* c, int code, const std::string& msg) {
    if (c) c->err = msg;
    throw Fail{code};
}

void hipchk(hbpc_ctx* c, hipError_t e, const char* what) {
    if (e != hipSuccess) set_err(c, HBPC_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

template <typename T> T* dalloc(hbpc_ctx* c, size_t count) {
    if (count == 0) count = 1;
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, count * sizeof(T));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        set_err(c, HBPC_ERR_OOM, "device allocation of " + std::to_string(count * sizeof(T)) + " bytes failed");
    }
    return (T*)p;
}

void dfree(void* p) {
    if (p) (void)hipFree(p);
}

double now_ms() {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}
}  // namespace

// Named host ranges (roctx, seen by rocprofv3 --marker-trace) around the phases of a step: the
// step, each predictor stage, each corrector sweep, each stage solve (or pair of them) and each
// BJ_ext build.  Launches are asynchronous, but every Arnoldi iteration waits for its results, so
// a range's host time follows the GPU work it enqueues.
struct PhaseRange {
    explicit PhaseRange(const char* name) { roctxRangePushA(name); }
    ~PhaseRange() { roctxRangePop(); }
    PhaseRange(const PhaseRange&) = delete;
    PhaseRange& operator=(const PhaseRange&) = delete;
};

// ------------------------------------------------------------------ kernel timing
static const char* KC_NAMES[KC_COUNT] = {"trace",    "r1",        "r2",   "res",  "jvp", "kcol",   "pcpre",
                                         "bj_apply", "bj_invert", "mdot", "gemv", "vec", "gs_dot", "gs_update",
                                         "lin",      "mlp_feat",  "mlp_gemm", "mlp_vec", "ns_grad", "bj_apply4"};

// record a launch of class cls (all classes, or only c->prof_only when that is >= 0)
static long prof_begin(hbpc_ctx* c, int cls) {
    if (!c->prof || (c->prof_only >= 0 && cls != c->prof_only)) return -1;
    size_t i = c->ev_used;
    if (c->ev.size() < 2 * (i + 1)) {
        hipEvent_t a, b;
        if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return -1;
        c->ev.push_back(a);
        c->ev.push_back(b);
        c->ev_class.push_back(0);
        c->ev_bytes.push_back(0);
        c->ev_flops.push_back(0);
    }
    (void)hipEventRecord(c->ev[2 * i], c->stream);
    c->ev_used = i + 1;
    return (long)i;
}

static void prof_end(hbpc_ctx* c, long i, int cls, double bytes, double flops = 0.0) {
    if (i < 0) return;
    (void)hipEventRecord(c->ev[2 * i + 1], c->stream);
    c->ev_class[i] = cls;
    c->ev_bytes[i] = bytes;
    c->ev_flops[i] = flops;
}

static void prof_resolve(hbpc_ctx* c) {
    if (c->ev_used == 0) return;
    (void)hipStreamSynchronize(c->stream);
    for (size_t i = 0; i < c->ev_used; ++i) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, c->ev[2 * i], c->ev[2 * i + 1]) != hipSuccess) continue;
        int k = c->ev_class[i];
        c->kp_launch[k] += 1;
        c->kp_ms[k] += ms;
        c->kp_bytes[k] += c->ev_bytes[i];
        c->kp_flops[k] += c->ev_flops[i];
    }
    c->ev_used = 0;
}

// ------------------------------------------------------------------ operator wrappers
LaunchReq op_req(hbpc_ctx* c, int op) {
    LaunchReq r;
    std::memset(&r, 0, sizeof(r));
    r.op = op;
    r.stream = c->stream;
    return r;
}

int op_launch(hbpc_ctx* c, const LaunchReq& r, int f32) {
    const double esz = f32 ? 4.0 : 8.0, n = (double)c->ndof;
    int cls = KC_VEC;
    double bytes = 0.0;
    switch (r.op) {
    case OPK_TRACE: cls = KC_TRACE; bytes = (n + (double)c->tsz) * esz * (r.col > 1 ? r.col : 1); break;
    case OPK_R1: cls = KC_R1; bytes = 2 * n * esz; break;
    case OPK_R2: cls = KC_R2; bytes = 3 * n * esz; break;
    case OPK_RES: cls = KC_RES; bytes = 5 * n * esz; break;
    case OPK_JVP:
    case OPK_JVP_NOHESS: cls = KC_JVP; bytes = 6 * n * esz; break;
    case OPK_KCOL: cls = KC_KCOL; bytes = (double)(r.e_end - r.e_begin) * c->NE * (8.0 + c->NE * 8.0); break;
    case OPK_KHCOL: cls = KC_KCOL; bytes = (double)(r.e_end - r.e_begin) * c->NE * (16.0 + c->NE * 16.0); break;
    case OPK_PCPRE: cls = KC_PCPRE; bytes = 5 * n * esz; break;
    case OPK_LINLOC: cls = KC_LIN; bytes = 4 * n * esz; break;
    }
    if (r.pair) {
        if (c->ns) set_err(c, HBPC_ERR_UNSUPPORTED, "paired operator launch with BR2 lifting");
        bytes *= 2;
    }
    if (c->ns && r.op != OPK_TRACE) {
        // BR2: the face gradients of this op's jet over the whole mesh first (neighbour data of
        // the operator kernel), then the operator with them
        LaunchReq ra = r;
        ra.aux = 1;
        ra.e_begin = 0;
        ra.e_end = 0;
        for (int j = 0; j < 4; ++j) ra.nsg[j] = c->nsg[f32][j];
        long pa = prof_begin(c, KC_NSGRAD);
        hipError_t ea = c->launch(c->geom, ra, f32);
        prof_end(c, pa, KC_NSGRAD, bytes);
        if (ea != hipSuccess) set_err(c, HBPC_ERR_HIP, std::string("face-gradient kernel launch: ") + hipGetErrorString(ea));
        LaunchReq rm = r;
        for (int j = 0; j < 4; ++j) rm.nsg[j] = c->nsg[f32][j];
        long pi = prof_begin(c, cls);
        hipError_t e = c->launch(c->geom, rm, f32);
        prof_end(c, pi, cls, bytes);
        if (e != hipSuccess) set_err(c, HBPC_ERR_HIP, std::string("operator kernel launch: ") + hipGetErrorString(e));
        return 0;
    }
    long pi = prof_begin(c, cls);
    hipError_t e = c->launch(c->geom, r, f32);
    prof_end(c, pi, cls, bytes);
    if (e != hipSuccess) set_err(c, HBPC_ERR_HIP, std::string("operator kernel launch: ") + hipGetErrorString(e));
    return 0;
}

// traces of nf consecutive fields (x: nf x ndof, tr: nf x tsz)
static void op_trace(hbpc_ctx* c, const void* x, void* tr, int f32, int nf = 1) {
    LaunchReq r = op_req(c, OPK_TRACE);
    r.fld[0] = x;
    r.out[0] = tr;
    r.col = nf;
    op_launch(c, r, f32);
}

// BR1: traces of the lifted gradient of field x (needs the traces of x) into slot `slot`
static const void* op_lift(hbpc_ctx* c, const void* x, const void* trx, int slot, int f32) {
    if (!c->visc) return nullptr;
    LaunchReq r = op_req(c, OPK_LIFT);
    r.fld[0] = x;
    r.trc[0] = trx;
    r.out[0] = c->qtr[f32][slot];
    op_launch(c, r, f32);
    return c->qtr[f32][slot];
}

// R1(w) -> out; traces of w written to trw (FP64)
static void op_r1(hbpc_ctx* c, const double* w, double* out, double* trw) {
    op_trace(c, w, trw, 0);
    LaunchReq r = op_req(c, OPK_R1);
    r.fld[0] = w;
    r.trc[0] = trw;
    r.qtr[0] = op_lift(c, w, trw, 0, 0);
    r.out[0] = out;
    op_launch(c, r, 0);
}

// R2(w, sigma) -> out with given traces of w and sigma
static void op_r2_tr(hbpc_ctx* c, const double* w, const double* s, const double* trw, const double* trs,
                     double* out) {
    LaunchReq r = op_req(c, OPK_R2);
    r.fld[0] = w;
    r.fld[1] = s;
    r.trc[0] = trw;
    r.trc[1] = trs;
    r.qtr[0] = op_lift(c, w, trw, 0, 0);
    r.qtr[1] = op_lift(c, s, trs, 1, 0);
    r.out[0] = out;
    op_launch(c, r, 0);
}

// R1 and R2(w, R1(w)) of a stage value
static void op_r1r2(hbpc_ctx* c, const double* w, double* r1, double* r2) {
    op_r1(c, w, r1, c->trw);
    op_trace(c, r1, c->trs, 0);
    op_r2_tr(c, w, r1, c->trw, c->trs, r2);
}

// G(X) with the traces of X in trw/trs (FP64)
static void op_res(hbpc_ctx* c, const double* X, const double* b, double a1dt, double bc, double* G,
                   const double* trw, const double* trs);
static void op_res(hbpc_ctx* c, const double* X, const double* b, double a1dt, double bc, double* G) {
    op_res(c, X, b, a1dt, bc, G, c->trw, c->trs);
}
static void op_res(hbpc_ctx* c, const double* X, const double* b, double a1dt, double bc, double* G,
                   const double* trw, const double* trs) {
    LaunchReq r = op_req(c, OPK_RES);
    r.fld[0] = X;
    r.fld[1] = X + c->ndof;
    r.fld[2] = b;
    r.trc[0] = trw;
    r.trc[1] = trs;
    r.qtr[0] = op_lift(c, X, trw, 0, 0);
    r.qtr[1] = op_lift(c, X + c->ndof, trs, 1, 0);
    r.out[0] = G;
    r.out[1] = G + c->ndof;
    r.c0 = a1dt;
    r.c1 = bc;
    op_launch(c, r, 0);
}

// linearised JVP in precision f32: state (w, s) with traces (trw, trs), input dX, output Y (2 ndof)
static void op_jvp(hbpc_ctx* c, const void* w, const void* s, const void* trw, const void* trs, const void* dX,
                   void* Y, double a1dt, double bc, int f32, int hess) {
    size_t esz = f32 ? 4 : 8;
    const char* dx = (const char*)dX;
    char* y = (char*)Y;
    void* t1 = f32 ? (void*)c->trd1_32 : (void*)c->trd1;
    void* t2 = f32 ? (void*)c->trd2_32 : (void*)c->trd2;
    op_trace(c, dx, t1, f32, 2);   // t2 = t1 + tsz
    LaunchReq r = op_req(c, hess ? OPK_JVP : OPK_JVP_NOHESS);
    r.fld[0] = w;
    r.fld[1] = s;
    r.fld[2] = dx;
    r.fld[3] = dx + c->ndof * esz;
    r.trc[0] = trw;
    r.trc[1] = trs;
    r.trc[2] = t1;
    r.trc[3] = t2;
    r.qtr[0] = op_lift(c, w, trw, 0, f32);
    r.qtr[1] = op_lift(c, s, trs, 1, f32);
    r.qtr[2] = op_lift(c, dx, t1, 2, f32);
    r.qtr[3] = op_lift(c, dx + c->ndof * esz, t2, 3, f32);
    r.out[0] = y;
    r.out[1] = y + c->ndof * esz;
    r.c0 = a1dt;
    r.c1 = bc;
    op_launch(c, r, f32);
}

// J X_i for two systems in one trace launch and one operator launch (equations without BR1/BR2
// lifting): system i at state (w_i, s_i) with traces (trw_i, trs_i), its dX_i traced into tx_i
// (2 tsz values of the Krylov precision)
static void op_jvp_pair(hbpc_ctx* c, const void* const* w, const void* const* s, const void* const* trw,
                        const void* const* trs, const void* const* dX, void* const* Y, void* const* tx, double a1dt,
                        double bc, int f32, int hess) {
    if (c->visc || c->ns) set_err(c, HBPC_ERR_UNSUPPORTED, "paired JVP launch with lifting");
    const size_t esz = f32 ? 4 : 8, tb = c->tsz * esz;
    LaunchReq t[2], r[2];
    for (int i = 0; i < 2; ++i) {
        t[i] = op_req(c, OPK_TRACE);
        t[i].fld[0] = dX[i];
        t[i].out[0] = tx[i];
        t[i].col = 2;
        r[i] = op_req(c, hess ? OPK_JVP : OPK_JVP_NOHESS);
        r[i].fld[0] = w[i];
        r[i].fld[1] = s[i];
        r[i].fld[2] = dX[i];
        r[i].fld[3] = (const char*)dX[i] + c->ndof * esz;
        r[i].trc[0] = trw[i];
        r[i].trc[1] = trs[i];
        r[i].trc[2] = tx[i];
        r[i].trc[3] = (const char*)tx[i] + tb;
        r[i].out[0] = Y[i];
        r[i].out[1] = (char*)Y[i] + c->ndof * esz;
        r[i].c0 = a1dt;
        r[i].c1 = bc;
    }
    t[0].pair = &t[1];
    r[0].pair = &r[1];
    op_launch(c, t[0], f32);
    op_launch(c, r[0], f32);
}

static void status_reset(hbpc_ctx* c) { hipchk(c, hipMemsetAsync(c->dstatus, 0, sizeof(int), c->stream), "memset"); }

static int status_read(hbpc_ctx* c) {
    int h = 0;
    hipchk(c, hipMemcpyAsync(&h, c->dstatus, sizeof(int), hipMemcpyDeviceToHost, c->stream), "copy status");
    hipchk(c, hipStreamSynchronize(c->stream), "sync");
    return h;
}

// ||x||_2 (FP64 or FP32 vector of length n), synchronising
static double dnorm(hbpc_ctx* c, const void* x, size_t n, int f32) {
    // own result slots after the two Arnoldi slots (an iteration in flight may be writing those)
    hipchk(c, blas_mdot(x, 0, 1, x, n, f32, c->part, c->dres + c->arn_len, c->stream), "norm");
    hipchk(c, hipMemcpyAsync(c->hres + 2 * c->arn_len, c->dres + c->arn_len, sizeof(double), hipMemcpyDeviceToHost,
                             c->stream),
           "copy");
    hipchk(c, hipStreamSynchronize(c->stream), "sync");
    return std::sqrt(c->hres[2 * c->arn_len]);
}

// ------------------------------------------------------------------ BJ_ext
// BJ_ext blocks at w, or with sigma given the BJ^H_ext blocks at (w, sigma) (Sec. 3.2.3)
static void pc_build(hbpc_ctx* c, const double* w, const double* sigma, double a1dt, double bc, int f32) {
    PhaseRange range("BJ_ext build");
    const bool hess = sigma != nullptr;
    double t0 = now_ms();
    if (c->NE > 1024) set_err(c, HBPC_ERR_UNSUPPORTED, "BJ_ext supports element blocks up to 1024 unknowns");
    const int type = f32 ? (c->prm.pc_half ? 2 : 1) : 0;
    const size_t esz = type == 2 ? 2 : (type == 1 ? 4 : 8);
    void*& S = c->Sinv_slot[c->cur_slot];
    if (!S || c->sinv_type_slot[c->cur_slot] != type) {
        dfree(S);
        S = nullptr;
        c->slot_valid[c->cur_slot] = 0;
        size_t cnt = (size_t)c->nE * c->NE * c->NE;
        S = (void*)dalloc<char>(c, cnt * esz);
        c->sinv_type_slot[c->cur_slot] = type;
    }
    c->Sinv = S;
    c->sinv_f32 = f32;
    c->sinv_type = type;
    if (!c->KT) c->KT = dalloc<double>(c, c->kt_chunk * c->NE * c->NE);
    if (hess && !c->HT) c->HT = dalloc<double>(c, c->kt_chunk * c->NE * c->NE);
    op_trace(c, w, c->trw, 0);
    if (hess) op_trace(c, sigma, c->trs, 0);
    status_reset(c);
    for (size_t eb = 0; eb < (size_t)c->nE; eb += c->kt_chunk) {
        size_t ee = std::min((size_t)c->nE, eb + c->kt_chunk);
        {
            LaunchReq r = op_req(c, hess ? OPK_KHCOL : OPK_KCOL);   // all NE columns in one launch
            r.fld[0] = w;
            r.trc[0] = c->trw;
            r.qtr[0] = op_lift(c, w, c->trw, 0, 0);
            r.out[0] = c->KT;
            if (hess) {
                // the lifted gradient of sigma only reaches the e_s part, which is not written
                r.fld[1] = sigma;
                r.trc[1] = c->trs;
                r.out[1] = c->HT;
            }
            r.e_begin = (int)eb;
            r.e_end = (int)ee;
            op_launch(c, r, 0);
        }
        long pi = prof_begin(c, KC_BJINV);
        hipchk(c, bj_invert(c->KT, hess ? c->HT : nullptr, (char*)c->Sinv + eb * c->NE * c->NE * esz, type, c->NE,
                            (int)(ee - eb), a1dt, bc, c->dstatus, c->stream),
               "bj_invert");
        const double ne = c->NE, cnt = (double)(ee - eb);
        prof_end(c, pi, KC_BJINV, cnt * ne * ne * ((hess ? 16.0 : 8.0) + esz), cnt * 4.0 * ne * ne * ne);
    }
    if (status_read(c)) set_err(c, HBPC_ERR_NONFINITE, "BJ_ext: singular or non-finite element block");
    c->pc_a1dt = a1dt;
    c->pc_bc = bc;
    c->pc_valid = 1;
    c->pc_hess = hess;
    c->slot_hess[c->cur_slot] = hess;
    c->slot_a1dt[c->cur_slot] = a1dt;
    c->slot_bc[c->cur_slot] = bc;
    c->slot_valid[c->cur_slot] = 1;
    c->st.pc_builds++;
    c->st.t_pc_build_ms += now_ms() - t0;
}

// make S^-1 slot `slot` the active one (BJ_ext apply reads c->Sinv, c->pc_a1dt, c->pc_bc)
static void pc_use_slot(hbpc_ctx* c, int slot) {
    c->cur_slot = slot;
    c->Sinv = c->Sinv_slot[slot];
    c->sinv_type = c->sinv_type_slot[slot];
    c->sinv_f32 = c->sinv_type != 0;
    c->pc_a1dt = c->slot_a1dt[slot];
    c->pc_bc = c->slot_bc[slot];
    c->pc_valid = c->slot_valid[slot];
    c->pc_hess = c->slot_hess[slot];
}

static void op_lin_local(hbpc_ctx* c, const void* w, const void* trw, const void* s, const void* x, double coef,
                         void* out, int f32);

// Y = P^-1 X in precision f32; the linearisation state (w, traces) in the same precision
static void pc_apply(hbpc_ctx* c, const void* w, const void* trw, const void* X, void* Y, int f32) {
    size_t esz = f32 ? 4 : 8;
    char* kv = (char*)c->kv;   // a | c
    if (c->pc_hess) {
        // BJ^H_ext: S^-1 no longer commutes with K; y = S^-1 (vw - bcoef K vs), P^-1 X = (y, vs + K y)
        const char* vs = (const char*)X + c->ndof * esz;
        char* ys = (char*)Y + c->ndof * esz;
        op_lin_local(c, w, trw, vs, X, -c->pc_bc, kv, f32);
        long pi = prof_begin(c, KC_BJAPPLY);
        hipchk(c, bj_apply(c->Sinv, c->sinv_type, kv, kv, Y, ys, f32, c->NE, c->nE, c->stream), "bj_apply");
        prof_end(c, pi, KC_BJAPPLY,
                 (double)c->nE * c->NE * c->NE * (c->sinv_type == 2 ? 2.0 : (c->sinv_type == 1 ? 4.0 : 8.0)) +
                     4.0 * c->ndof * esz);
        op_lin_local(c, w, trw, Y, vs, 1.0, ys, f32);
        return;
    }
    LaunchReq r = op_req(c, OPK_PCPRE);
    r.fld[0] = w;
    r.fld[1] = X;
    r.fld[2] = (const char*)X + c->ndof * esz;
    r.trc[0] = trw;
    r.qtr[0] = op_lift(c, w, trw, 0, f32);
    r.out[0] = kv;
    r.out[1] = kv + c->ndof * esz;
    r.c0 = c->pc_a1dt;
    r.c1 = c->pc_bc;
    op_launch(c, r, f32);
    long pi = prof_begin(c, KC_BJAPPLY);
    hipchk(c, bj_apply(c->Sinv, c->sinv_type, kv, kv + c->ndof * esz, Y, (char*)Y + c->ndof * esz, f32, c->NE, c->nE,
                       c->stream),
           "bj_apply");
    prof_end(c, pi, KC_BJAPPLY,
             (double)c->nE * c->NE * c->NE * (c->sinv_type == 2 ? 2.0 : (c->sinv_type == 1 ? 4.0 : 8.0)) +
                 4.0 * c->ndof * esz);
}

// ------------------------------------------------------------------ learned preconditioner
// out = x + coef K(w) s with the element-local Jacobian K of BJ_ext (traces of w given)
static void op_lin_local(hbpc_ctx* c, const void* w, const void* trw, const void* s, const void* x, double coef,
                         void* out, int f32) {
    LaunchReq r = op_req(c, OPK_LINLOC);
    r.fld[0] = w;
    r.fld[1] = s;
    r.fld[2] = x;
    r.trc[0] = trw;
    r.qtr[0] = op_lift(c, w, trw, 0, f32);
    r.out[0] = out;
    r.c0 = coef;
    op_launch(c, r, f32);
}

struct MlpView {
    const float *W1r, *W1w, *b1, *W2r, *W2w, *b2, *W3;
};

// parameter blocks in the order W1r (n_r x H), W1w (n_w x H), b1, W2r, W2w, b2, W3 (H x NE)
template <typename P> static void mlp_blocks(const hbpc_ctx* c, P* th, P** out) {
    const size_t nr = c->mlp_nr, nw = c->mlp_nin - c->mlp_nr, H = c->mlp_H, no = c->NE;
    out[0] = th;
    out[1] = out[0] + nr * H;
    out[2] = out[1] + nw * H;
    out[3] = out[2] + H;
    out[4] = out[3] + H * H;
    out[5] = out[4] + H * H;
    out[6] = out[5] + H;
}

static MlpView mlp_view(const hbpc_ctx* c, const float* th) {
    const float* b[7];
    mlp_blocks(c, th, b);
    return MlpView{b[0], b[1], b[2], b[3], b[4], b[5], b[6]};
}

// C = A B (+bias, relu) (.* mask | .* (mask > 0)) (+= C)
static void mlp_gemm_p(hbpc_ctx* c, const float* A, long long a_r, long long a_c, const float* B, long long b_r,
                       long long b_c, float* C, long long ldc, const float* bias, const float* mask, int mask_mul,
                       int M, int N, int K, int relu, int bf16, int accumulate = 0) {
    long pi = prof_begin(c, KC_GEMM);
    // a weight operand is read from the BF16 copy of the parameters
    const uint16_t* B16 = nullptr;
    if (bf16 && B >= c->theta && B < c->theta + c->mlp_np) B16 = c->theta16 + (B - c->theta);
    hipchk(c, mlp_gemm(A, a_r, a_c, B, B16, b_r, b_c, C, ldc, bias, mask, mask ? ldc : 0, mask_mul, M, N, K, relu,
                       accumulate, bf16, c->gemm_ws, c->gemm_ws_floats, c->stream),
           "mlp gemm");
    prof_end(c, pi, KC_GEMM, 4.0 * ((double)M * K + (double)K * N + (double)M * N * (mask ? 2 : 1)),
             2.0 * M * N * K);
}

static void mlp_ew(hbpc_ctx* c, hipError_t e, double bytes) {
    hipchk(c, e, "mlp elementwise");
    (void)bytes;
}

// state gates of `rows` feature rows: G1 = relu(Xw W1w + b1), G2 = relu(G1 W2w + b2)
static void mlp_gates(hbpc_ctx* c, const float* X, int rows, float* G1, float* G2, int bf16) {
    const int ni = c->mlp_nin, nr = c->mlp_nr, H = c->mlp_H;
    MlpView p = mlp_view(c, c->theta);
    mlp_gemm_p(c, X + nr, ni, 1, p.W1w, H, 1, G1, H, p.b1, nullptr, 0, rows, H, ni - nr, 1, bf16);
    mlp_gemm_p(c, G1, H, 1, p.W2w, H, 1, G2, H, p.b2, nullptr, 0, rows, H, H, 1, bf16);
}

// residual path with the gates given: H1 = (Xr W1r) .* G1, H2 = (H1 W2r) .* G2, Y = H2 W3
static void mlp_residual_path(hbpc_ctx* c, const float* X, int rows, const float* G1, const float* G2, float* H1,
                              float* H2, float* Y, int bf16) {
    const int ni = c->mlp_nin, nr = c->mlp_nr, H = c->mlp_H, no = c->NE;
    MlpView p = mlp_view(c, c->theta);
    mlp_gemm_p(c, X, ni, 1, p.W1r, H, 1, H1, H, nullptr, G1, 1, rows, H, nr, 0, bf16);
    mlp_gemm_p(c, H1, H, 1, p.W2r, H, 1, H2, H, nullptr, G2, 1, rows, H, H, 0, bf16);
    mlp_gemm_p(c, H2, H, 1, p.W3, no, 1, Y, no, nullptr, nullptr, 0, rows, no, H, 0, bf16);
}

// training buffers: per row 10 H + 2 NE (activations, gradients) + n_in + NE (gathered batch)
static void mlp_train_alloc(hbpc_ctx* c, int rows) {
    if (rows <= c->tr_rows) return;
    dfree(c->tr_buf);
    c->tr_buf = nullptr;
    c->tr_rows = 0;
    const size_t per = 10 * (size_t)c->mlp_H + 3 * (size_t)c->NE + (size_t)c->mlp_nin;
    c->tr_buf = dalloc<float>(c, per * rows);
    c->tr_rows = rows;
}

// Sum of squared errors of f(X) - T over rows x NE added to *sse (device); gradient of
// the mean squared error into grad.  Work space: the training buffers.
static void mlp_loss_grad_dev(hbpc_ctx* c, const float* X, const float* T, int rows, float* grad, double* sse,
                              int bf16) {
    const int ni = c->mlp_nin, nr = c->mlp_nr, nw = ni - nr, H = c->mlp_H, no = c->NE;
    mlp_train_alloc(c, rows);
    const size_t RH = (size_t)rows * H;
    float* g1 = c->tr_buf;
    float* g2 = g1 + RH;
    float* a1 = g2 + RH;
    float* h1 = a1 + RH;
    float* a2 = h1 + RH;
    float* h2 = a2 + RH;
    float* D1 = h2 + RH;
    float* D2 = D1 + RH;
    float* D3 = D2 + RH;
    float* D4 = D3 + RH;
    float* Y = D4 + RH;
    float* dY = Y + (size_t)rows * no;
    MlpView p = mlp_view(c, c->theta);
    float* gb[7];
    mlp_blocks(c, grad, gb);
    const long long nH = (long long)RH;
    // forward, keeping the pre-gate products
    mlp_gates(c, X, rows, g1, g2, bf16);
    mlp_gemm_p(c, X, ni, 1, p.W1r, H, 1, a1, H, nullptr, nullptr, 0, rows, H, nr, 0, bf16);
    mlp_ew(c, mlp_ew_mul(a1, g1, h1, nH, c->stream), 12.0 * nH);
    mlp_gemm_p(c, h1, H, 1, p.W2r, H, 1, a2, H, nullptr, nullptr, 0, rows, H, H, 0, bf16);
    mlp_ew(c, mlp_ew_mul(a2, g2, h2, nH, c->stream), 12.0 * nH);
    mlp_gemm_p(c, h2, H, 1, p.W3, no, 1, Y, no, nullptr, nullptr, 0, rows, no, H, 0, bf16);
    // loss
    const long long n = (long long)rows * no;
    const int nblk = (int)std::min<long long>(64, (n + 255) / 256);
    long pi = prof_begin(c, KC_MLPV);
    hipchk(c, mlp_mse_grad(Y, T, dY, n, (float)(1.0 / (double)n), c->part, nblk, c->stream), "mse");
    hipchk(c, mlp_sum_parts(c->part, nblk, sse, c->stream), "mse");
    prof_end(c, pi, KC_MLPV, 12.0 * n);
    // y = h2 W3
    mlp_gemm_p(c, h2, 1, H, dY, no, 1, gb[6], no, nullptr, nullptr, 0, H, no, rows, 0, bf16);
    mlp_gemm_p(c, dY, no, 1, p.W3, 1, no, D1, H, nullptr, nullptr, 0, rows, H, no, 0, bf16);   // dh2
    // h2 = a2 .* g2: da2 -> D2, dz2 = dh2 .* a2 .* (g2 > 0) -> D3
    mlp_ew(c, mlp_ew_split(D1, g2, a2, D2, D3, nH, 1, c->stream), 20.0 * nH);
    // a2 = h1 W2r
    mlp_gemm_p(c, h1, 1, H, D2, H, 1, gb[3], H, nullptr, nullptr, 0, H, H, rows, 0, bf16);
    mlp_gemm_p(c, D2, H, 1, p.W2r, 1, H, D1, H, nullptr, nullptr, 0, rows, H, H, 0, bf16);    // dh1
    // h1 = a1 .* g1: da1 -> D2, dh1 .* a1 -> D4
    mlp_ew(c, mlp_ew_split(D1, g1, a1, D2, D4, nH, 0, c->stream), 20.0 * nH);
    // a1 = Xr W1r
    mlp_gemm_p(c, X, 1, ni, D2, H, 1, gb[0], H, nullptr, nullptr, 0, nr, H, rows, 0, bf16);
    // g2 = relu(g1 W2w + b2)
    mlp_gemm_p(c, g1, 1, H, D3, H, 1, gb[4], H, nullptr, nullptr, 0, H, H, rows, 0, bf16);
    hipchk(c, mlp_colsum(D3, H, rows, H, gb[5], c->stream), "colsum");
    mlp_gemm_p(c, D3, H, 1, p.W2w, 1, H, D4, H, nullptr, nullptr, 0, rows, H, H, 0, bf16, 1);   // dg1 += dz2 W2w^T
    // g1 = relu(Xw W1w + b1)
    mlp_ew(c, mlp_ew_relu_mask(D4, g1, nH, c->stream), 12.0 * nH);
    mlp_gemm_p(c, X + nr, 1, ni, D4, H, 1, gb[1], H, nullptr, nullptr, 0, nw, H, rows, 0, bf16);
    hipchk(c, mlp_colsum(D4, H, rows, H, gb[2], c->stream), "colsum");
}

static void mlp_adam_dev(hbpc_ctx* c, const float* grad, double lr, double b1, double b2, double eps) {
    c->adam_t++;
    long pi = prof_begin(c, KC_MLPV);
    hipchk(c, mlp_adam(c->theta, c->theta16, grad, c->adam_m, c->adam_v, (long long)c->mlp_np, (float)lr, (float)b1, (float)b2,
                       (float)eps, c->adam_t, c->stream),
           "adam");
    prof_end(c, pi, KC_MLPV, 20.0 * c->mlp_np);
}

static void lpc_buffers(hbpc_ctx* c) {
    if (c->ap_X) return;
    const size_t nE = c->nE;
    c->ap_X = dalloc<float>(c, nE * c->mlp_nin);
    c->ap_G1 = dalloc<float>(c, nE * c->mlp_H);
    c->ap_G2 = dalloc<float>(c, nE * c->mlp_H);
    c->ap_H1 = dalloc<float>(c, nE * c->mlp_H);
    c->ap_H2 = dalloc<float>(c, nE * c->mlp_H);
    c->ap_Y = dalloc<float>(c, nE * c->NE);
    c->ap_s = dalloc<float>(c, nE);
}

// part: 1 residual tiles (+scale, targets), 2 state tiles and coefficients, 3 both
static void features_p(hbpc_ctx* c, const void* rt, const void* w, const void* dw, int f32, const int* elems,
                       int count, double a1dt, double bc, float* X, float* T, float* scale, int part) {
    long pi = prof_begin(c, KC_FEAT);
    // the step coefficients enter as logarithms: O(1) values that tell the stage solves apart
    const float la = (float)std::log(std::max(a1dt, 1e-300)), lb = (float)std::log(std::max(bc, 1e-300));
    hipchk(c, mlp_features(rt, w, dw, f32, elems, count, c->D, c->geom.nel, c->NE, la, lb, X, T, scale, part,
                           c->stream),
           "mlp features");
    const double esz = f32 ? 4.0 : 8.0;
    const double tiles = (double)c->mlp_nr;   // patch values per field
    double bytes = 0.0;
    if (part & 1) bytes += tiles * (esz + 4.0) + 4.0 + (dw ? c->NE * (esz + 4.0) : 0.0);
    if (part & 2) bytes += tiles * (esz + 4.0) + 8.0;
    prof_end(c, pi, KC_FEAT, (double)count * bytes);
}

// gates of the learned preconditioner at linearisation state w (precision f32) and the coefficients
static void lpc_prepare(hbpc_ctx* c, const void* w, int f32, double a1dt, double bc, float* G1 = nullptr,
                        float* G2 = nullptr) {
    lpc_buffers(c);
    c->pc_a1dt = a1dt;
    c->pc_bc = bc;
    const int bf16 = c->prm.mlp_precision == HBPC_MLP_BF16;
    features_p(c, nullptr, w, nullptr, f32, nullptr, c->nE, a1dt, bc, c->ap_X, nullptr, nullptr, 2);
    mlp_gates(c, c->ap_X, c->nE, G1 ? G1 : c->ap_G1, G2 ? G2 : c->ap_G2, bf16);
}

// Y = P^-1 X with the learned preconditioner, vectors in precision f32, linearisation state w
// (traces trw) and gates G1, G2 (default: the context's) as given to the last lpc_prepare for w
static void lpc_apply(hbpc_ctx* c, const void* w, const void* trw, const void* Xv, void* Y, int f32,
                      const float* G1 = nullptr, const float* G2 = nullptr) {
    const size_t esz = f32 ? 4 : 8, n = c->ndof;
    const char* vw = (const char*)Xv;
    const char* vs = vw + n * esz;
    char* yw = (char*)Y;
    char* ys = yw + n * esz;
    void* rt = c->kv;
    const int bf16 = c->prm.mlp_precision == HBPC_MLP_BF16;
    op_lin_local(c, w, trw, vs, vw, -c->pc_bc, rt, f32);   // rt = vw - bcoef K vs
    features_p(c, rt, w, nullptr, f32, nullptr, c->nE, c->pc_a1dt, c->pc_bc, c->ap_X, nullptr, c->ap_s, 1);
    mlp_residual_path(c, c->ap_X, c->nE, G1 ? G1 : c->ap_G1, G2 ? G2 : c->ap_G2, c->ap_H1, c->ap_H2, c->ap_Y, bf16);
    long pi = prof_begin(c, KC_MLPV);
    hipchk(c, mlp_rescale(c->ap_Y, c->ap_s, yw, f32, (long long)n, c->NE, c->stream), "mlp rescale");
    prof_end(c, pi, KC_MLPV, (double)n * (4.0 + esz) + 4.0 * c->nE);
    op_lin_local(c, w, trw, yw, vs, 1.0, ys, f32);          // ys = vs + K yw
}

// splitmix64 (Steele, Lea & Flood 2014): state advanced by the golden-ratio increment
static unsigned long long splitmix64(unsigned long long& x) {
    unsigned long long z = (x += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// first k entries of a Fisher-Yates shuffle of 0..n-1
static void draw_distinct(unsigned long long& state, int n, int k, std::vector<int>& out) {
    std::vector<int> p(n);
    for (int i = 0; i < n; ++i) p[i] = i;
    for (int i = 0; i < k; ++i) {
        int j = i + (int)(splitmix64(state) % (unsigned long long)(n - i));
        std::swap(p[i], p[j]);
    }
    out.assign(p.begin(), p.begin() + k);
}

// Training pairs from a Krylov vector v of a BJ_ext solve and z = P^-1 v: for k elements drawn with
// splitmix64, the features of rt = vw - bcoef K vs and the w block of z, i.e. the element solve
// S_e^-1 rt_e of BJ_ext (precision f32, linearisation state w with traces trw)
static void lpc_collect_krylov(hbpc_ctx* c, const void* w, const void* trw, const void* v, const void* z,
                               double a1dt, double bc, int f32) {
    const size_t esz = f32 ? 4 : 8, n = c->ndof;
    int k = (int)std::min<size_t>((size_t)c->col_per, c->col_cap - c->col_count);
    k = std::min(k, c->nE);
    if (k <= 0) return;
    const void* target = z;
    if (c->col_source == HBPC_MLP_PAIRS_RANDOM) {
        // target dw: standard normal values; rt = S dw = dw - a1dt K dw + bcoef K (K dw), the
        // element-local Schur operator of BJ_ext applied exactly
        void* dw = c->tmp[2];
        void* t = c->tmp[3];
        char* rt = (char*)c->kv;
        char* x = rt + n * esz;
        hipchk(c, mlp_randn(dw, f32, (long long)n, c->col_seed ^ (0xD1B54A32D192ED03ull * ++c->col_draws),
                            c->stream),
               "randn");
        hipchk(c, hipMemsetAsync(x, 0, n * esz, c->stream), "memset");
        op_lin_local(c, w, trw, dw, x, 1.0, t, f32);                          // t = K dw
        hipchk(c, blas_axpby(1.0, dw, f32, 0.0, x, f32, n, c->stream), "copy");
        hipchk(c, blas_axpby(-a1dt, t, f32, 1.0, x, f32, n, c->stream), "axpby");   // x = dw - a1dt t
        op_lin_local(c, w, trw, t, x, bc, rt, f32);                           // rt = x + bcoef K t
        target = dw;
    } else {
        op_lin_local(c, w, trw, (const char*)v + n * esz, v, -bc, c->kv, f32);
    }
    std::vector<int> el;
    draw_distinct(c->col_seed, c->nE, k, el);
    hipchk(c, hipMemcpyAsync(c->col_elems, el.data(), (size_t)k * sizeof(int), hipMemcpyHostToDevice, c->stream),
           "copy");
    features_p(c, c->kv, w, target, f32, c->col_elems, k, a1dt, bc, c->col_X + c->col_count * c->mlp_nin,
               c->col_T + c->col_count * c->NE, nullptr, 3);
    hipchk(c, hipStreamSynchronize(c->stream), "sync");   // el is host memory of this frame
    c->col_count += k;
    c->st.mlp_samples += k;
}

// Training pairs from the Newton correction just computed: rhs = -G, dX (FP64), state X with traces trw
static void lpc_collect(hbpc_ctx* c, double a1dt, double bc, const double* X = nullptr, const double* trw = nullptr,
                        const double* rhs = nullptr, const double* dX = nullptr) {
    if (!c->col_X || c->col_count >= c->col_cap || c->col_source != HBPC_MLP_PAIRS_NEWTON) return;
    if (!X) {   // the single-stage system
        X = c->X;
        trw = c->trw;
        rhs = c->rhs;
        dX = c->dX;
    }
    const size_t n = c->ndof;
    int k = (int)std::min<size_t>((size_t)c->col_per, c->col_cap - c->col_count);
    k = std::min(k, c->nE);
    if (k <= 0) return;
    double* rt = (double*)c->kv;
    op_lin_local(c, X, trw, rhs + n, rhs, -bc, rt, 0);   // rt = rhs_w - bcoef K rhs_s
    std::vector<int> el;
    draw_distinct(c->col_seed, c->nE, k, el);
    hipchk(c, hipMemcpyAsync(c->col_elems, el.data(), (size_t)k * sizeof(int), hipMemcpyHostToDevice, c->stream),
           "copy");
    features_p(c, rt, X, dX, 0, c->col_elems, k, a1dt, bc, c->col_X + c->col_count * c->mlp_nin,
               c->col_T + c->col_count * c->NE, nullptr, 3);
    hipchk(c, hipStreamSynchronize(c->stream), "sync");   // el is host memory of this frame
    c->col_count += k;
    c->st.mlp_samples += k;
}

// ------------------------------------------------------------------ FD JVP (Eq. MatrixFree_nonlinear), FP64
static void fd_alloc(hbpc_ctx* c) {
    for (int i = 0; i < 6; ++i)
        if (!c->fd[i]) c->fd[i] = dalloc<double>(c, c->ndof);
}

// requires fd[0] = R1(w), fd[1] = R2(w, sigma) precomputed; trw/trs traces of (w, sigma)
static void op_jvp_fd(hbpc_ctx* c, const double* w, const double* s, const double* dX, double* Y, double a1dt,
                      double bc) {
    const size_t n = c->ndof;
    const double* dw = dX;
    const double* ds = dX + n;
    const double emach = 2.220446049250313e-16;
    double nw = dnorm(c, dw, n, 0), ns = dnorm(c, ds, n, 0);
    double* T1 = c->fd[2];
    double* T3 = c->fd[3];
    double* T2 = c->fd[4];
    double* wp = c->fd[5];
    double* trp = c->trd1;   // traces of the perturbed state
    double* trq = c->trd2;
    double* r1p = (double*)c->kv;   // 3 n scratch in FP64 mode only
    double* r2p = r1p + n;
    double* sp = r2p + n;
    if (nw > 0) {
        double ew = std::sqrt(emach) / (c->geom.eps * nw);
        hipchk(c, blas_lincomb2(1.0, w, ew, dw, wp, n, c->stream), "fd");
        op_r1(c, wp, r1p, trp);                     // R1(w + ew dw); traces of wp in trp
        hipchk(c, blas_lincomb2(1.0 / ew, r1p, -1.0 / ew, c->fd[0], T1, n, c->stream), "fd");
        op_r2_tr(c, wp, s, trp, c->trs, r2p);       // R2(w + ew dw, sigma)
        hipchk(c, blas_lincomb2(1.0 / ew, r2p, -1.0 / ew, c->fd[1], T3, n, c->stream), "fd");
    } else {
        hipchk(c, hipMemsetAsync(T1, 0, n * 8, c->stream), "memset");
        hipchk(c, hipMemsetAsync(T3, 0, n * 8, c->stream), "memset");
    }
    if (ns > 0) {
        double es = std::sqrt(emach) / (c->geom.eps * ns);
        hipchk(c, blas_lincomb2(1.0, s, es, ds, sp, n, c->stream), "fd");
        op_trace(c, sp, trq, 0);
        op_r2_tr(c, w, sp, c->trw, trq, r2p);       // R2(w, sigma + es dsigma)
        hipchk(c, blas_lincomb2(1.0 / es, r2p, -1.0 / es, c->fd[1], T2, n, c->stream), "fd");
    } else {
        hipchk(c, hipMemsetAsync(T2, 0, n * 8, c->stream), "memset");
    }
    // Yw = dw - a1dt T1 + bc (T3 + T2);  Ys = ds - T1
    hipchk(c, blas_axpby(1.0, dw, 0, 0.0, Y, 0, n, c->stream), "fd");
    hipchk(c, blas_axpby(-a1dt, T1, 0, 1.0, Y, 0, n, c->stream), "fd");
    if (c->prm.hessian) hipchk(c, blas_axpby(bc, T3, 0, 1.0, Y, 0, n, c->stream), "fd");
    hipchk(c, blas_axpby(bc, T2, 0, 1.0, Y, 0, n, c->stream), "fd");
    hipchk(c, blas_lincomb2(1.0, ds, -1.0, T1, Y + n, n, c->stream), "fd");
}

// ------------------------------------------------------------------ FGMRES
// Solve J dX = rhs (FP64 rhs, FP64 dX accumulation) with Krylov vectors in precision f32.
// The linearisation state is c->X (FP64) / c->X32 (FP32) with traces trw/trs (and *_32).
static int fgmres(hbpc_ctx* c, const double* rhs, double* dX, double a1dt, double bc, int f32) {
    const size_t n2 = c->n2;
    const size_t esz = f32 ? 4 : 8;
    const int m = c->prm.gmres_restart;
    const int maxit = c->prm.gmres_maxit;
    const double rtol = c->prm.gmres_rtol;
    const int use_pc = c->prm.precond != HBPC_PC_NONE;
    const int fd = c->prm.jvp_mode == HBPC_JVP_FD && !f32;
    char* V = (char*)c->V;
    char* Z = (char*)c->Z;
    const void* w = f32 ? (const void*)c->X32 : (const void*)c->X;
    const void* s = f32 ? (const void*)(c->X32 + c->ndof) : (const void*)(c->X + c->ndof);
    const void* trw = f32 ? (const void*)c->trw32 : (const void*)c->trw;
    const void* trs = f32 ? (const void*)c->trs32 : (const void*)c->trs;
    auto Vj = [&](int j) { return (void*)(V + (size_t)j * n2 * esz); };
    auto Zj = [&](int j) { return (void*)(Z + (size_t)j * n2 * esz); };
    auto jvp = [&](const void* x, void* y) {
        if (fd) op_jvp_fd(c, (const double*)w, (const double*)s, (const double*)x, (double*)y, a1dt, bc);
        else op_jvp(c, w, s, trw, trs, x, y, a1dt, bc, f32, c->prm.hessian);
    };
    if (fd) {   // R1(w), R2(w, sigma) of the linearisation state
        fd_alloc(c);
        op_r1(c, c->X, c->fd[0], c->trd1);
        op_r2_tr(c, c->X, c->X + c->ndof, c->trw, c->trs, c->fd[1]);
    }
    hipchk(c, hipMemsetAsync(dX, 0, n2 * 8, c->stream), "memset");
    const double beta0 = dnorm(c, rhs, n2, 0);
    if (!std::isfinite(beta0)) set_err(c, HBPC_ERR_NONFINITE, "non-finite Newton residual");
    if (beta0 == 0.0) return 0;
    // residual vector r (precision f32) in V_0 slot; first cycle r = rhs
    hipchk(c, blas_axpby(1.0, rhs, 0, 0.0, Vj(0), f32, n2, c->stream), "copy");
    if (c->prm.precond == HBPC_PC_LEARNED_GUESS && c->lpc_active) {
        // initial guess z = N(rhs) (the network is linear in the residual): r = rhs - J z, kept
        // when it is smaller than rhs
        void* z = Zj(0);
        void* u = Vj(1);
        lpc_apply(c, w, trw, Vj(0), z, f32);
        jvp(z, u);
        hipchk(c, blas_axpby(-1.0, u, f32, 1.0, Vj(0), f32, n2, c->stream), "guess residual");
        const double nr = dnorm(c, Vj(0), n2, f32);
        if (std::isfinite(nr) && nr < beta0) {
            hipchk(c, blas_axpby(1.0, z, f32, 1.0, dX, 0, n2, c->stream), "guess");
            if (nr <= rtol * beta0) return 0;
        } else {
            c->st.pc_fallbacks++;
            hipchk(c, blas_axpby(1.0, rhs, 0, 0.0, Vj(0), f32, n2, c->stream), "copy");
        }
        if (c->verbose)
            std::fprintf(stderr, "[hbpc] learned initial guess: |r| %.3e -> %.3e\n", beta0, nr);
    }
    int total = 0, cycle = 0;
    std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1), y(m);
    auto Hc = [&](int i, int j) -> double& { return H[(size_t)i * m + j]; };
    for (;;) {
        double beta = dnorm(c, Vj(0), n2, f32);
        if (!std::isfinite(beta)) set_err(c, HBPC_ERR_NONFINITE, "non-finite Krylov residual");
        hipchk(c, blas_axpby(1.0 / beta, Vj(0), f32, 0.0, Vj(0), f32, n2, c->stream), "scale");
        std::fill(g.begin(), g.end(), 0.0);
        g[0] = beta;
        bool converged = false, bad_pc = false;
        int k = 0;
        const double beta_cycle = beta;
        const int learned = c->prm.precond == HBPC_PC_LEARNED && c->lpc_active;
        // network for z_0 only, in the first cycle (v_0 = the normalised Newton residual)
        const int net_first = c->prm.precond == HBPC_PC_LEARNED_FIRST && c->lpc_active && cycle == 0;
        // the network's first cycle of the solve may be a shorter probe, judged at the same mean rate
        const int probe = c->prm.pc_probe_its;
        const int mc = learned && cycle == 0 && probe > 0 && probe < m ? probe : m;
        const double fall = mc < m ? std::pow(c->prm.pc_fallback, (double)mc / m) : c->prm.pc_fallback;
        // Arnoldi iteration j, enqueued without waiting for the host: z_j = P^-1 v_j, u = J z_j,
        // classical Gram-Schmidt twice against V_0..V_j, the second pass taken from the Gram
        // matrix G = V^T V (V^T (u - V h1) = h1 - G h1, so one pass over V gives V^T u and the
        // new column of G, and one update subtracts V (2 h1 - G h1)), v_{j+1} = u / ||u||,
        // results (h, ||u||^2) copied to host slot j % 2
        auto enqueue = [&](int j) {
            void* zj = use_pc ? Zj(j) : Vj(j);
            if (learned || (net_first && j == 0)) lpc_apply(c, w, trw, Vj(j), zj, f32);
            else if (use_pc) pc_apply(c, w, trw, Vj(j), zj, f32);
            if (!learned && c->col_X && c->col_source != HBPC_MLP_PAIRS_NEWTON &&
                (use_pc || c->col_source == HBPC_MLP_PAIRS_RANDOM) && c->col_count < c->col_cap &&
                (total + j) % c->col_every == 0)
                lpc_collect_krylov(c, w, trw, Vj(j), zj, a1dt, bc, f32);
            void* u = Vj(j + 1);
            jvp(zj, u);
            const size_t R = (size_t)c->m_alloc + 1;
            double* h1 = c->dres;              // V^T u, then (adjacent) g = V^T v_j: 2 (j + 1) <= 2 R
            double* hn = c->dres + 2 * R;      // ||u - V h||^2
            double* h = c->dres + 2 * R + 4;   // two-pass coefficients, j + 1 <= R
            const double vb = (double)n2 * esz;
            long pi = prof_begin(c, KC_GSDOT);
            hipchk(c, blas_gs_gram(V, n2, j + 1, u, Vj(j), n2, f32, c->part, h1, h1 + (j + 1), c->dgram, m + 1, h,
                                   c->dcount, c->stream),
                   "gs dot");
            prof_end(c, pi, KC_GSDOT, (j + 3) * vb);
            pi = prof_begin(c, KC_GSUPD);
            hipchk(c, blas_gs_update_normalize(V, n2, j + 1, h, u, n2, f32, c->part, hn, c->stream), "gs update");
            prof_end(c, pi, KC_GSUPD, (j + 5) * vb);
            hipchk(c, hipMemcpyAsync(c->hres + c->arn_len * (j & 1), c->dres, (3 * R + 4) * sizeof(double),
                                     hipMemcpyDeviceToHost, c->stream),
                   "copy");
            hipchk(c, hipEventRecord(c->arn_ev[j & 1], c->stream), "event");
        };
        enqueue(0);
        for (int j = 0; j < mc; ++j) {
            // the next iteration goes to the GPU before this one's results are read (it is
            // discarded if this one ends the cycle)
            if (j + 1 < mc && total + 1 < maxit) enqueue(j + 1);
            hipchk(c, hipEventSynchronize(c->arn_ev[j & 1]), "sync");
            const double* hr = c->hres + c->arn_len * (j & 1);
            const size_t R = (size_t)c->m_alloc + 1;
            for (int i = 0; i <= j; ++i) Hc(i, j) = hr[2 * R + 4 + i];
            double hnrm = std::sqrt(hr[2 * R]);
            Hc(j + 1, j) = hnrm;
            if (!std::isfinite(hnrm)) {
                // a non-finite learned-preconditioner output: drop column j and fall back
                if ((learned || (net_first && j == 0)) && c->prm.pc_fallback > 0) {
                    bad_pc = true;
                    k = j;
                    break;
                }
                set_err(c, HBPC_ERR_NONFINITE, "non-finite Arnoldi vector");
            }
            for (int i = 0; i < j; ++i) {
                double t = cs[i] * Hc(i, j) + sn[i] * Hc(i + 1, j);
                Hc(i + 1, j) = -sn[i] * Hc(i, j) + cs[i] * Hc(i + 1, j);
                Hc(i, j) = t;
            }
            double den = std::hypot(Hc(j, j), Hc(j + 1, j));
            cs[j] = Hc(j, j) / den;
            sn[j] = Hc(j + 1, j) / den;
            Hc(j, j) = den;
            Hc(j + 1, j) = 0.0;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            ++total;
            k = j + 1;
            if (std::fabs(g[j + 1]) <= rtol * beta0) { converged = true; break; }
            if (total >= maxit) break;
            if (hnrm == 0.0) { converged = true; break; }
        }
        // y = H^-1 g (upper triangular), dX += Z y
        for (int i = k - 1; i >= 0; --i) {
            double t = g[i];
            for (int l = i + 1; l < k; ++l) t -= Hc(i, l) * y[l];
            y[i] = t / Hc(i, i);
        }
        if (k > 0) hipchk(c, blas_gemv_add(use_pc ? Z : V, f32, n2, k, y.data(), dX, 0, n2, c->stream), "update");
        if (converged) return total;
        if (total >= maxit) {
            set_err(c, HBPC_ERR_GMRES, "GMRES did not reach eps_G within " + std::to_string(maxit) + " iterations");
        }
        // learned preconditioner: BJ_ext takes over after a poor cycle or a non-finite output; the
        // cycle's correction is dropped and BJ_ext starts from the right-hand side (keeping it
        // left residuals on which BJ_ext needed more iterations than on the original one)
        if ((learned || net_first) && c->prm.pc_fallback > 0 &&
            (bad_pc || (learned && std::fabs(g[k]) > fall * beta_cycle))) {
            c->lpc_active = 0;
            c->st.pc_fallbacks++;
            if (c->verbose)
                std::fprintf(stderr, "[hbpc] learned preconditioner -> BJ_ext (%s, cycle %d reduced |r| by %.3e)\n",
                             bad_pc ? "non-finite" : "slow", cycle, std::fabs(g[k]) / beta_cycle);
            // (built already for the first-direction form, or kept for this stage)
            if (learned && !c->pc_kept) pc_build(c, c->X, nullptr, a1dt, bc, f32);
            hipchk(c, hipMemsetAsync(dX, 0, n2 * 8, c->stream), "memset");
            hipchk(c, blas_axpby(1.0, rhs, 0, 0.0, Vj(0), f32, n2, c->stream), "copy");
            ++cycle;
            continue;
        }
        ++cycle;
        // restart: r = rhs - J dX, computed in precision f32 in V_0
        void* xw = Vj(1);   // dX in precision f32
        hipchk(c, blas_axpby(1.0, dX, 0, 0.0, xw, f32, n2, c->stream), "cast");
        jvp(xw, Vj(0));
        hipchk(c, blas_axpby(1.0, rhs, 0, -1.0, Vj(0), f32, n2, c->stream), "residual");
    }
}

// ------------------------------------------------------------------ Newton
static void state_traces(hbpc_ctx* c, int mixed) {
    op_trace(c, c->X, c->trw, 0);
    op_trace(c, c->X + c->ndof, c->trs, 0);
    if (mixed) {
        hipchk(c, blas_axpby(1.0, c->X, 0, 0.0, c->X32, 1, c->n2, c->stream), "cast");
        op_trace(c, c->X32, c->trw32, 1);
        op_trace(c, c->X32 + c->ndof, c->trs32, 1);
    }
}

// solve g(W) = b for W (a1dt = alpha1 dt, bc = alpha2 dt^2/2), initial guess `guess`; W -> out.
// keep_pc: BJ_ext blocks of the active slot built for the same coefficients and precision are used
// as they are.
static void newton_solve(hbpc_ctx* c, const double* b, double a1dt, double bc, const double* guess, double* out,
                         bool keep_pc = false) {
    PhaseRange range("stage solve");
    const size_t n = c->ndof;
    const int mixed = c->prm.precision == HBPC_MIXED;
    double* X = c->X;
    hipchk(c, hipMemcpyAsync(X, guess, n * 8, hipMemcpyDeviceToDevice, c->stream), "copy");
    op_r1(c, X, X + n, c->trw);              // sigma^0 = R1(guess)
    state_traces(c, 0);
    op_res(c, X, b, a1dt, bc, c->G);
    const double n0 = dnorm(c, c->G, c->n2, 0);
    if (!std::isfinite(n0)) set_err(c, HBPC_ERR_NONFINITE, "non-finite residual at the Newton initial guess");
    const double nw0 = dnorm(c, X, n, 0);   // ||w^0||, scale of the rounding-floor test
    double nr_prev = n0;
    int its = 0, gits = 0;
    const int sidx = c->cur_solve;
    if (n0 > 1e-14 * std::sqrt((double)c->n2)) {
        if (mixed) state_traces(c, 1);
        const int pck = c->prm.precond;
        const int first = pck == HBPC_PC_LEARNED_FIRST || pck == HBPC_PC_LEARNED_GUESS;
        const double* sig_h = pck == HBPC_PC_BJEXT_H ? X + n : nullptr;   // BJ^H_ext: at (w, sigma)
        const bool kept = keep_pc && c->pc_valid && c->pc_a1dt == a1dt && c->pc_bc == bc && c->sinv_f32 == mixed &&
                          c->pc_hess == (sig_h != nullptr);
        c->pc_kept = kept;
        if ((pck == HBPC_PC_BJEXT || pck == HBPC_PC_BJEXT_H || first) && !kept) pc_build(c, X, sig_h, a1dt, bc, mixed);
        if (pck == HBPC_PC_LEARNED || first) {
            if (!c->mlp_ready) set_err(c, HBPC_ERR_ARG, "learned preconditioner without parameters");
            c->lpc_active = 1;
        }
        for (;;) {
            ++its;
            const int bj = pck == HBPC_PC_BJEXT || pck == HBPC_PC_BJEXT_H || first ||
                           (pck == HBPC_PC_LEARNED && !c->lpc_active);
            if (bj && c->prm.pc_rebuild == HBPC_PC_PER_NEWTON_IT && its > 1) pc_build(c, X, sig_h, a1dt, bc, mixed);
            // learned: gates at the current linearisation state
            if ((pck == HBPC_PC_LEARNED || first) && c->lpc_active)
                lpc_prepare(c, mixed ? (const void*)c->X32 : (const void*)X, mixed, a1dt, bc);
            hipchk(c, blas_axpby(-1.0, c->G, 0, 0.0, c->rhs, 0, c->n2, c->stream), "rhs");
            double tg = now_ms();
            gits += fgmres(c, c->rhs, c->dX, a1dt, bc, mixed);
            c->st.t_gmres_ms += now_ms() - tg;
            lpc_collect(c, a1dt, bc);
            hipchk(c, blas_axpby(1.0, c->dX, 0, 1.0, X, 0, c->n2, c->stream), "update");
            state_traces(c, mixed);
            op_res(c, X, b, a1dt, bc, c->G);
            double nr = dnorm(c, c->G, c->n2, 0);
            double ndw = dnorm(c, c->dX, n, 0);
            if (c->verbose)
                std::fprintf(stderr, "[hbpc] solve %d newton %d |G| %.6e (|G0| %.6e) |dw| %.3e gmres %d\n", sidx, its,
                             nr, n0, ndw, gits);
            if (!std::isfinite(nr)) set_err(c, HBPC_ERR_NONFINITE, "non-finite Newton residual");
            // absolute criterion per coefficient (RMS of dw), see hbpc_params.newton_atol_dw
            if (nr <= c->prm.newton_rtol * n0 || ndw <= c->prm.newton_atol_dw * std::sqrt((double)n)) break;
            // rounding floor: the residual stopped falling and the update is at the state's rounding level
            if (its >= 2 && nr > 0.5 * nr_prev && ndw <= 1e-12 * nw0) {
                c->st.newton_floor_stops++;
                break;
            }
            nr_prev = nr;
            if (its >= c->prm.newton_maxit)
                set_err(c, HBPC_ERR_NEWTON,
                        "Newton did not converge within " + std::to_string(c->prm.newton_maxit) + " iterations");
        }
    }
    hipchk(c, hipMemcpyAsync(out, X, n * 8, hipMemcpyDeviceToDevice, c->stream), "copy");
    if (sidx < HBPC_MAX_SOLVES) {
        c->st.newton_per_solve[sidx] = its;
        c->st.gmres_per_solve[sidx] = gits;
    }
    c->st.newton_its += its;
    c->st.gmres_its += gits;
    c->cur_solve++;
    c->st.n_solves = c->cur_solve;
}

// ------------------------------------------------------------------ paired corrector stage solves
// HBPC_PC_PAIRED: two corrector stage equations of a sweep (independent, Alg. 1) solved side by
// side.  Newton and FGMRES iterations advance in lock step; per iteration the PCPRE products of
// both systems, one pass of bj_apply over the shared S^-1 for the four right-hand sides, then per
// system the JVP at its own state and the Gram-Schmidt passes, with the next iteration enqueued
// before the host reads this one's results.  A system that converges drops out while the other
// goes on.  With the learned preconditioner each system starts its stage solve on the network
// (gates at its own state) and falls back to the shared BJ_ext blocks on its own.  Stopping
// rules as in fgmres() and newton_solve().
static StageSys sys_ctx(hbpc_ctx* c) {
    StageSys S;
    S.X = c->X;
    S.G = c->G;
    S.dX = c->dX;
    S.rhs = c->rhs;
    S.b = c->b;
    S.trw = c->trw;
    S.trs = c->trs;
    S.X32 = c->X32;
    S.trw32 = c->trw32;
    S.trs32 = c->trs32;
    S.V = (char*)c->V;
    S.Z = (char*)c->Z;
    S.kv = c->kv;
    S.part = c->part;
    S.dres = c->dres;
    S.dgram = c->dgram;
    S.hres = c->hres;
    S.dcount = c->dcount;
    S.lpc = 0;
    S.G1 = c->ap_G1;
    S.G2 = c->ap_G2;
    S.trd1 = c->trd1;
    S.trd1_32 = c->trd1_32;
    return S;
}

static void pair_alloc(hbpc_ctx* c) {
    StageSys& P = c->pair;
    if (P.X) return;
    const size_t n = c->ndof, n2 = c->n2, esz = c->kr_f32 ? 4 : 8;
    P.X = dalloc<double>(c, n2);
    P.G = dalloc<double>(c, n2);
    P.dX = dalloc<double>(c, n2);
    P.rhs = dalloc<double>(c, n2);
    P.b = dalloc<double>(c, n);
    P.trw = dalloc<double>(c, c->tsz);
    P.trs = dalloc<double>(c, c->tsz);
    P.X32 = dalloc<float>(c, n2);
    P.trw32 = dalloc<float>(c, c->tsz);
    P.trs32 = dalloc<float>(c, c->tsz);
    P.V = dalloc<char>(c, (size_t)(c->m_alloc + 1) * n2 * esz);
    P.Z = dalloc<char>(c, (size_t)c->m_alloc * n2 * esz);
    P.kv = dalloc<char>(c, n2 * esz);
    P.part = dalloc<double>(c, (size_t)blas_mdot_grid(n2) * (2 * (c->m_alloc + 1) + 2) + 64);
    P.dres = dalloc<double>(c, c->arn_len + 64);
    P.dgram = dalloc<double>(c, (size_t)(c->m_alloc + 1) * (c->m_alloc + 1));
    P.dcount = dalloc<unsigned>(c, 4);
    hipchk(c, hipMemset(P.dcount, 0, 4 * sizeof(unsigned)), "memset");
    void* h = nullptr;
    hipchk(c, hipHostMalloc(&h, (2 * c->arn_len + 64) * sizeof(double)), "hipHostMalloc");
    P.hres = (double*)h;
    P.trd1 = dalloc<double>(c, 2 * c->tsz);
    P.trd1_32 = dalloc<float>(c, 2 * c->tsz);
}

static void pair_free(hbpc_ctx* c) {
    StageSys& P = c->pair;
    void* bufs[] = {P.X, P.G, P.dX, P.rhs, P.b, P.trw, P.trs, P.X32, P.trw32, P.trs32, P.V, P.Z, P.kv,
                    P.part, P.dres, P.dgram, P.dcount, P.G1, P.G2, P.trd1, P.trd1_32};
    for (void* q : bufs) dfree(q);
    if (P.hres) (void)hipHostFree(P.hres);
    std::memset(&P, 0, sizeof(P));
}

static void sys_traces(hbpc_ctx* c, const StageSys& S, int mixed) {
    op_trace(c, S.X, S.trw, 0);
    op_trace(c, S.X + c->ndof, S.trs, 0);
    if (mixed) {
        hipchk(c, blas_axpby(1.0, S.X, 0, 0.0, S.X32, 1, c->n2, c->stream), "cast");
        op_trace(c, S.X32, S.trw32, 1);
        op_trace(c, S.X32 + c->ndof, S.trs32, 1);
    }
}

// PCPRE products a = vw - bcoef K vs, c = vs + K (vw - a1dt vs) of one Krylov vector into kv
static void pcpre_into(hbpc_ctx* c, const void* w, const void* trw, const void* X, void* kv, int f32) {
    const size_t esz = f32 ? 4 : 8;
    LaunchReq r = op_req(c, OPK_PCPRE);
    r.fld[0] = w;
    r.fld[1] = X;
    r.fld[2] = (const char*)X + c->ndof * esz;
    r.trc[0] = trw;
    r.qtr[0] = op_lift(c, w, trw, 0, f32);
    r.out[0] = kv;
    r.out[1] = (char*)kv + c->ndof * esz;
    r.c0 = c->pc_a1dt;
    r.c1 = c->pc_bc;
    op_launch(c, r, f32);
}

// the PCPRE products of two systems' Krylov vectors in one launch (no lifting)
static void pcpre_pair(hbpc_ctx* c, const void* const* w, const void* const* trw, const void* const* X,
                       void* const* kv, int f32) {
    const size_t esz = f32 ? 4 : 8;
    LaunchReq r[2];
    for (int i = 0; i < 2; ++i) {
        r[i] = op_req(c, OPK_PCPRE);
        r[i].fld[0] = w[i];
        r[i].fld[1] = X[i];
        r[i].fld[2] = (const char*)X[i] + c->ndof * esz;
        r[i].trc[0] = trw[i];
        r[i].out[0] = kv[i];
        r[i].out[1] = (char*)kv[i] + c->ndof * esz;
        r[i].c0 = c->pc_a1dt;
        r[i].c1 = c->pc_bc;
    }
    r[0].pair = &r[1];
    op_launch(c, r[0], f32);
}

static void fgmres_pair(hbpc_ctx* c, StageSys* S, int* active, double a1dt, double bc, int f32, int* its) {
    const size_t n2 = c->n2, n = c->ndof, esz = f32 ? 4 : 8;
    const int m = c->prm.gmres_restart, maxit = c->prm.gmres_maxit;
    const double rtol = c->prm.gmres_rtol;
    const size_t R = (size_t)c->m_alloc + 1;
    // per system: the current restart cycle (H, Givens rotations, g), iteration j to be read next
    // and e to be enqueued next (e - j <= 2), and a generation number that marks iterations of
    // a cycle that has ended (they are discarded)
    struct Cyc {
        std::vector<double> H, cs, sn, g, y;
        int j = 0, e = 0, total = 0, cycle = 0, gen = 0, mc = 0;
        double beta0 = 0.0, beta_cyc = 0.0, fall = 0.0;
        bool on = false, learned = false;
    } cy[2];
    auto Vj = [&](int i, int j) { return (void*)(S[i].V + (size_t)j * n2 * esz); };
    auto Zj = [&](int i, int j) { return (void*)(S[i].Z + (size_t)j * n2 * esz); };
    auto wst = [&](int i) { return f32 ? (const void*)S[i].X32 : (const void*)S[i].X; };
    auto sst = [&](int i) { return f32 ? (const void*)(S[i].X32 + n) : (const void*)(S[i].X + n); };
    auto tw = [&](int i) { return f32 ? (const void*)S[i].trw32 : (const void*)S[i].trw; };
    auto ts = [&](int i) { return f32 ? (const void*)S[i].trs32 : (const void*)S[i].trs; };
    // a new cycle of system i from the residual in V_0: normalise, reset the Hessenberg data; the
    // learned preconditioner's first cycle may be a shorter probe, judged at the same mean rate
    auto start_cycle = [&](int i) {
        const double beta = dnorm(c, Vj(i, 0), n2, f32);
        if (!std::isfinite(beta)) set_err(c, HBPC_ERR_NONFINITE, "non-finite Krylov residual");
        hipchk(c, blas_axpby(1.0 / beta, Vj(i, 0), f32, 0.0, Vj(i, 0), f32, n2, c->stream), "scale");
        Cyc& C = cy[i];
        C.H.assign((size_t)(m + 1) * m, 0.0);
        C.cs.assign(m, 0.0);
        C.sn.assign(m, 0.0);
        C.g.assign(m + 1, 0.0);
        C.y.assign(m, 0.0);
        C.g[0] = beta;
        C.beta_cyc = beta;
        C.j = C.e = 0;
        C.gen++;
        C.learned = S[i].lpc != 0;
        const int probe = c->prm.pc_probe_its;
        C.mc = C.learned && C.cycle == 0 && probe > 0 && probe < m ? probe : m;
        C.fall = C.mc < m ? std::pow(c->prm.pc_fallback, (double)C.mc / m) : c->prm.pc_fallback;
    };
    for (int i = 0; i < 2; ++i) {
        its[i] = 0;
        if (!active[i]) continue;
        hipchk(c, hipMemsetAsync(S[i].dX, 0, n2 * 8, c->stream), "memset");
        cy[i].beta0 = dnorm(c, S[i].rhs, n2, 0);
        if (!std::isfinite(cy[i].beta0)) set_err(c, HBPC_ERR_NONFINITE, "non-finite Newton residual");
        if (cy[i].beta0 == 0.0) continue;
        hipchk(c, blas_axpby(1.0, S[i].rhs, 0, 0.0, Vj(i, 0), f32, n2, c->stream), "copy");
        start_cycle(i);
        cy[i].on = true;
    }
    // Round r: the next Arnoldi iteration of every system that has one, enqueued without
    // waiting for the host: z = P^-1 v (the learned systems first, since the network's work
    // space is the first system's PCPRE buffer; then the PCPRE products of the BJ_ext systems
    // and one pass of bj_apply over the shared blocks for all their right-hand sides), then per
    // system u = J z at its own state, the two Gram-Schmidt passes, results to host slot r % 2.
    struct Round {
        int cnt = 0, sys[2], it[2], gen[2];
    } rd[2];
    auto enqueue = [&](int r) {
        Round& Rr = rd[r & 1];
        Rr.cnt = 0;
        for (int i = 0; i < 2; ++i) {
            Cyc& C = cy[i];
            if (!C.on || C.e >= C.mc || C.total + (C.e - C.j) >= maxit) continue;
            Rr.sys[Rr.cnt] = i;
            Rr.it[Rr.cnt] = C.e++;
            Rr.gen[Rr.cnt++] = C.gen;
        }
        if (Rr.cnt == 0) return false;
        for (int q = 0; q < Rr.cnt; ++q) {
            const int i = Rr.sys[q], j = Rr.it[q];
            if (cy[i].learned) lpc_apply(c, wst(i), tw(i), Vj(i, j), Zj(i, j), f32, S[i].G1, S[i].G2);
        }
        const void* xs[4];
        void* ys[4];
        int nr = 0;
        const bool pre2 = Rr.cnt == 2 && !cy[Rr.sys[0]].learned && !cy[Rr.sys[1]].learned && !c->visc && !c->ns;
        if (pre2) {   // both systems' pre-products in one launch
            const void *w2[2], *t2[2], *x2[2];
            void* k2[2];
            for (int q = 0; q < 2; ++q) {
                const int i = Rr.sys[q];
                w2[q] = wst(i);
                t2[q] = tw(i);
                x2[q] = Vj(i, Rr.it[q]);
                k2[q] = S[i].kv;
            }
            pcpre_pair(c, w2, t2, x2, k2, f32);
        }
        for (int q = 0; q < Rr.cnt; ++q) {
            const int i = Rr.sys[q], j = Rr.it[q];
            if (cy[i].learned) continue;
            if (!pre2) pcpre_into(c, wst(i), tw(i), Vj(i, j), S[i].kv, f32);
            xs[nr] = S[i].kv;
            ys[nr++] = Zj(i, j);
            xs[nr] = (const char*)S[i].kv + n * esz;
            ys[nr++] = (char*)Zj(i, j) + n * esz;
        }
        if (nr > 0) {
            // one system: the plain apply (w and sigma halves); both: the four-right-hand-side kernel
            const int cls = nr > 2 ? KC_BJAPPLY4 : KC_BJAPPLY;
            long pi = prof_begin(c, cls);
            hipchk(c, bj_apply_n(c->Sinv, c->sinv_type, xs, ys, nr, f32, c->NE, c->nE, c->stream), "bj_apply");
            prof_end(c, pi, cls,
                     (double)c->nE * c->NE * c->NE * (c->sinv_type == 2 ? 2.0 : (c->sinv_type == 1 ? 4.0 : 8.0)) +
                         2.0 * nr * n * esz);
        }
        if (Rr.cnt == 2 && !c->visc && !c->ns) {
            // both systems: one trace and one JVP launch, one multi-dot (per chunk), one reduction,
            // one update and one normalisation launch for the two
            const void *w2[2], *s2[2], *tw2[2], *ts2[2], *dx2[2], *V2[2], *vj2[2], *u2c[2];
            void *y2[2], *tx2[2], *u2[2];
            int k2[2];
            double *part2[2], *h12[2], *G2[2], *h2[2], *hn2[2];
            unsigned* cnt2[2];
            double vb = 0.0, ub = 0.0;
            for (int q = 0; q < 2; ++q) {
                const int i = Rr.sys[q], j = Rr.it[q];
                w2[q] = wst(i);
                s2[q] = sst(i);
                tw2[q] = tw(i);
                ts2[q] = ts(i);
                dx2[q] = Zj(i, j);
                y2[q] = u2[q] = Vj(i, j + 1);
                u2c[q] = u2[q];
                tx2[q] = f32 ? (void*)S[i].trd1_32 : (void*)S[i].trd1;
                V2[q] = S[i].V;
                vj2[q] = Vj(i, j);
                k2[q] = j + 1;
                part2[q] = S[i].part;
                h12[q] = S[i].dres;
                hn2[q] = S[i].dres + 2 * R;
                h2[q] = S[i].dres + 2 * R + 4;
                G2[q] = S[i].dgram;
                cnt2[q] = S[i].dcount;
                vb += (j + 3) * (double)n2 * esz;
                ub += (j + 5) * (double)n2 * esz;
            }
            op_jvp_pair(c, w2, s2, tw2, ts2, dx2, y2, tx2, a1dt, bc, f32, c->prm.hessian);
            long pi = prof_begin(c, KC_GSDOT);
            hipchk(c, blas_gs_gram_n(2, V2, n2, k2, u2c, vj2, n2, f32, part2, h12, G2, m + 1, h2, cnt2, c->stream),
                   "gs dot");
            prof_end(c, pi, KC_GSDOT, vb);
            pi = prof_begin(c, KC_GSUPD);
            hipchk(c, blas_gs_update_normalize_n(2, V2, n2, k2, h2, u2, n2, f32, part2, hn2, c->stream), "gs update");
            prof_end(c, pi, KC_GSUPD, ub);
            for (int q = 0; q < 2; ++q) {
                const int i = Rr.sys[q];
                hipchk(c, hipMemcpyAsync(S[i].hres + c->arn_len * (r & 1), S[i].dres, (3 * R + 4) * sizeof(double),
                                         hipMemcpyDeviceToHost, c->stream),
                       "copy");
            }
            hipchk(c, hipEventRecord(c->arn_ev[r & 1], c->stream), "event");
            return true;
        }
        for (int q = 0; q < Rr.cnt; ++q) {
            const int i = Rr.sys[q], j = Rr.it[q];
            void* u = Vj(i, j + 1);
            op_jvp(c, wst(i), sst(i), tw(i), ts(i), Zj(i, j), u, a1dt, bc, f32, c->prm.hessian);
            double* h1 = S[i].dres;
            double* hn = S[i].dres + 2 * R;
            double* h = S[i].dres + 2 * R + 4;
            const double vb = (double)n2 * esz;
            long pi = prof_begin(c, KC_GSDOT);
            hipchk(c, blas_gs_gram(S[i].V, n2, j + 1, u, Vj(i, j), n2, f32, S[i].part, h1, h1 + (j + 1), S[i].dgram,
                                   m + 1, h, S[i].dcount, c->stream),
                   "gs dot");
            prof_end(c, pi, KC_GSDOT, (j + 3) * vb);
            pi = prof_begin(c, KC_GSUPD);
            hipchk(c, blas_gs_update_normalize(S[i].V, n2, j + 1, h, u, n2, f32, S[i].part, hn, c->stream),
                   "gs update");
            prof_end(c, pi, KC_GSUPD, (j + 5) * vb);
            hipchk(c, hipMemcpyAsync(S[i].hres + c->arn_len * (r & 1), S[i].dres, (3 * R + 4) * sizeof(double),
                                     hipMemcpyDeviceToHost, c->stream),
                   "copy");
        }
        hipchk(c, hipEventRecord(c->arn_ev[r & 1], c->stream), "event");
        return true;
    };
    // the host's part of iteration C.j of system i (slot: its results): Givens rotations, stopping
    // tests, and at the end of a cycle the update of dX, then a restart or the fallback to BJ_ext
    auto process = [&](int i, const double* hr) {
        Cyc& C = cy[i];
        const int j = C.j;
        auto Hc = [&](int a, int b) -> double& { return C.H[(size_t)a * m + b]; };
        for (int a = 0; a <= j; ++a) Hc(a, j) = hr[2 * R + 4 + a];
        const double hnrm = std::sqrt(hr[2 * R]);
        bool bad = false, conv = false;
        int k = j + 1;
        if (!std::isfinite(hnrm)) {
            // a non-finite learned-preconditioner output: drop column j and fall back
            if (!(C.learned && c->prm.pc_fallback > 0)) set_err(c, HBPC_ERR_NONFINITE, "non-finite Arnoldi vector");
            bad = true;
            k = j;
        } else {
            Hc(j + 1, j) = hnrm;
            for (int a = 0; a < j; ++a) {
                const double t = C.cs[a] * Hc(a, j) + C.sn[a] * Hc(a + 1, j);
                Hc(a + 1, j) = -C.sn[a] * Hc(a, j) + C.cs[a] * Hc(a + 1, j);
                Hc(a, j) = t;
            }
            const double den = std::hypot(Hc(j, j), Hc(j + 1, j));
            C.cs[j] = Hc(j, j) / den;
            C.sn[j] = Hc(j + 1, j) / den;
            Hc(j, j) = den;
            Hc(j + 1, j) = 0.0;
            C.g[j + 1] = -C.sn[j] * C.g[j];
            C.g[j] = C.cs[j] * C.g[j];
            ++C.total;
            C.j = j + 1;
            conv = std::fabs(C.g[j + 1]) <= rtol * C.beta0 || hnrm == 0.0;
            if (!conv && C.j < C.mc && C.total < maxit) return;
        }
        // end of the cycle: y = H^-1 g, dX += Z y
        for (int a = k - 1; a >= 0; --a) {
            double t = C.g[a];
            for (int l = a + 1; l < k; ++l) t -= Hc(a, l) * C.y[l];
            C.y[a] = t / Hc(a, a);
        }
        if (k > 0) hipchk(c, blas_gemv_add(S[i].Z, f32, n2, k, C.y.data(), S[i].dX, 0, n2, c->stream), "update");
        if (conv) {
            C.on = false;
            its[i] = C.total;
            return;
        }
        if (C.total >= maxit)
            set_err(c, HBPC_ERR_GMRES, "GMRES did not reach eps_G within " + std::to_string(maxit) + " iterations");
        ++C.cycle;
        if (C.learned && c->prm.pc_fallback > 0 && (bad || std::fabs(C.g[k]) > C.fall * C.beta_cyc)) {
            // BJ_ext takes over for the rest of this stage solve, from the right-hand side
            S[i].lpc = 0;
            c->st.pc_fallbacks++;
            if (c->verbose)
                std::fprintf(stderr, "[hbpc] (paired) learned preconditioner -> BJ_ext (%s, reduced |r| by %.3e)\n",
                             bad ? "non-finite" : "slow", std::fabs(C.g[k]) / C.beta_cyc);
            hipchk(c, hipMemsetAsync(S[i].dX, 0, n2 * 8, c->stream), "memset");
            hipchk(c, blas_axpby(1.0, S[i].rhs, 0, 0.0, Vj(i, 0), f32, n2, c->stream), "copy");
            start_cycle(i);
            return;
        }
        // restart: r = rhs - J dX in V_0
        void* xw = Vj(i, 1);
        hipchk(c, blas_axpby(1.0, S[i].dX, 0, 0.0, xw, f32, n2, c->stream), "cast");
        op_jvp(c, wst(i), sst(i), tw(i), ts(i), xw, Vj(i, 0), a1dt, bc, f32, c->prm.hessian);
        hipchk(c, blas_axpby(1.0, S[i].rhs, 0, -1.0, Vj(i, 0), f32, n2, c->stream), "residual");
        start_cycle(i);
    };
    auto any_on = [&]() { return cy[0].on || cy[1].on; };
    // one round in flight ahead of the host: round r + 1 is enqueued before round r's results
    // are read (its iterations are discarded where round r ends a cycle)
    int r = 0;
    bool pend = any_on() && enqueue(0);
    while (pend) {
        const bool ahead = enqueue(r + 1);
        hipchk(c, hipEventSynchronize(c->arn_ev[r & 1]), "sync");
        const Round& Rr = rd[r & 1];
        for (int q = 0; q < Rr.cnt; ++q) {
            const int i = Rr.sys[q];
            if (!cy[i].on || cy[i].gen != Rr.gen[q]) continue;
            process(i, S[i].hres + c->arn_len * (r & 1));
        }
        ++r;
        pend = ahead || (any_on() && enqueue(r));
    }
}

// Newton on two corrector stage equations g(W_i) = b_i side by side (see fgmres_pair); keep_pc: the
// active slot's blocks, built for the same coefficients and precision, are used as they are
static void newton_solve_pair(hbpc_ctx* c, const double* const* b, double a1dt, double bc,
                              const double* const* guess, double* const* out, bool keep_pc) {
    PhaseRange range("paired stage solves");
    pair_alloc(c);
    const size_t n = c->ndof;
    const int mixed = c->prm.precision == HBPC_MIXED;
    const bool learned = c->prm.precond == HBPC_PC_LEARNED;
    if (learned) {
        if (!c->mlp_ready) set_err(c, HBPC_ERR_ARG, "learned preconditioner without parameters");
        lpc_buffers(c);
        if (!c->pair.G1) {   // the second system's gates
            c->pair.G1 = dalloc<float>(c, (size_t)c->nE * c->mlp_H);
            c->pair.G2 = dalloc<float>(c, (size_t)c->nE * c->mlp_H);
        }
    }
    StageSys S[2] = {sys_ctx(c), c->pair};
    int active[2], its[2] = {0, 0}, gits[2] = {0, 0};
    double n0[2], nw0[2], nr_prev[2];
    for (int i = 0; i < 2; ++i) {
        hipchk(c, hipMemcpyAsync(S[i].X, guess[i], n * 8, hipMemcpyDeviceToDevice, c->stream), "copy");
        op_r1(c, S[i].X, S[i].X + n, S[i].trw);   // sigma^0 = R1(guess)
        sys_traces(c, S[i], 0);
        op_res(c, S[i].X, b[i], a1dt, bc, S[i].G, S[i].trw, S[i].trs);
        n0[i] = dnorm(c, S[i].G, c->n2, 0);
        if (!std::isfinite(n0[i])) set_err(c, HBPC_ERR_NONFINITE, "non-finite residual at the Newton initial guess");
        nw0[i] = dnorm(c, S[i].X, n, 0);
        nr_prev[i] = n0[i];
        active[i] = n0[i] > 1e-14 * std::sqrt((double)c->n2);
        if (active[i] && mixed) sys_traces(c, S[i], 1);
    }
    if (active[0] || active[1]) {
        const bool kept = keep_pc && c->pc_valid && c->pc_a1dt == a1dt && c->pc_bc == bc && c->sinv_f32 == mixed &&
                          !c->pc_hess;
        c->pc_kept = kept;
        if (!kept) pc_build(c, S[active[0] ? 0 : 1].X, nullptr, a1dt, bc, mixed);
        // learned: the network first in each stage solve, BJ_ext (the blocks above) after a fallback
        for (int i = 0; i < 2; ++i) S[i].lpc = learned && active[i];
    }
    while (active[0] || active[1]) {
        int run[2] = {active[0], active[1]};
        for (int i = 0; i < 2; ++i)
            if (run[i]) {
                ++its[i];
                // learned: gates at the system's current linearisation state
                if (S[i].lpc)
                    lpc_prepare(c, mixed ? (const void*)S[i].X32 : (const void*)S[i].X, mixed, a1dt, bc, S[i].G1,
                                S[i].G2);
                hipchk(c, blas_axpby(-1.0, S[i].G, 0, 0.0, S[i].rhs, 0, c->n2, c->stream), "rhs");
            }
        int git[2];
        const double tg = now_ms();
        fgmres_pair(c, S, run, a1dt, bc, mixed, git);
        c->st.t_gmres_ms += now_ms() - tg;
        for (int i = 0; i < 2; ++i) {
            if (!run[i]) continue;
            gits[i] += git[i];
            lpc_collect(c, a1dt, bc, S[i].X, S[i].trw, S[i].rhs, S[i].dX);
            hipchk(c, blas_axpby(1.0, S[i].dX, 0, 1.0, S[i].X, 0, c->n2, c->stream), "update");
            sys_traces(c, S[i], mixed);
            op_res(c, S[i].X, b[i], a1dt, bc, S[i].G, S[i].trw, S[i].trs);
            const double nr = dnorm(c, S[i].G, c->n2, 0);
            const double ndw = dnorm(c, S[i].dX, n, 0);
            if (c->verbose)
                std::fprintf(stderr, "[hbpc] solve %d (paired) newton %d |G| %.6e (|G0| %.6e) |dw| %.3e gmres %d\n",
                             c->cur_solve + i, its[i], nr, n0[i], ndw, gits[i]);
            if (!std::isfinite(nr)) set_err(c, HBPC_ERR_NONFINITE, "non-finite Newton residual");
            if (nr <= c->prm.newton_rtol * n0[i] || ndw <= c->prm.newton_atol_dw * std::sqrt((double)n)) {
                active[i] = 0;
            } else if (its[i] >= 2 && nr > 0.5 * nr_prev[i] && ndw <= 1e-12 * nw0[i]) {
                c->st.newton_floor_stops++;
                active[i] = 0;
            } else if (its[i] >= c->prm.newton_maxit) {
                set_err(c, HBPC_ERR_NEWTON,
                        "Newton did not converge within " + std::to_string(c->prm.newton_maxit) + " iterations");
            }
            nr_prev[i] = nr;
        }
    }
    for (int i = 0; i < 2; ++i) {
        hipchk(c, hipMemcpyAsync(out[i], S[i].X, n * 8, hipMemcpyDeviceToDevice, c->stream), "copy");
        const int sidx = c->cur_solve + i;
        if (sidx < HBPC_MAX_SOLVES) {
            c->st.newton_per_solve[sidx] = its[i];
            c->st.gmres_per_solve[sidx] = gits[i];
        }
        c->st.newton_its += its[i];
        c->st.gmres_its += gits[i];
    }
    c->cur_solve += 2;
    c->st.n_solves = c->cur_solve;
}

// ------------------------------------------------------------------ HBPC step (Algorithm 1)
static void hbpc_step_impl(hbpc_ctx* c, double* w_inout, double dt) {
    PhaseRange range("hbpc_step");
    Tab t;
    if (!tableau(c->prm.q, t)) set_err(c, HBPC_ERR_ARG, "q must be 4, 6 or 8");
    const int s = t.s;
    const size_t n = c->ndof;
    double** W = c->W;
    auto R1 = [&](int j) { return c->R1all + (size_t)j * n; };
    auto R2 = [&](int j) { return c->R2all + (size_t)j * n; };
    hipchk(c, hipMemcpyAsync(W[0], w_inout, n * 8, hipMemcpyDeviceToDevice, c->stream), "copy");
    op_r1r2(c, W[0], R1(0), R2(0));
    // blocks kept across steps: every slot is rebuilt on first use after pc_reuse_steps steps
    const bool across = c->prm.pc_rebuild == HBPC_PC_ACROSS_STEPS;
    if (across && c->pc_steps >= c->prm.pc_reuse_steps) {
        for (int i = 0; i < 4; ++i) c->slot_valid[i] = 0;
        c->pc_steps = 0;
    }
    // predictor: successive two-point Hermite-Birkhoff substeps
    for (int l = 1; l < s; ++l) {
        PhaseRange stage("predictor stage");
        double dc = t.c[l] - t.c[l - 1];
        double a1dt = dc / 2 * dt;
        double bc = dc * dc / 6 * dt * dt / 2;
        double coef1[4] = {0, 0, 0, 0}, coef2[4] = {0, 0, 0, 0};
        coef1[l - 1] = a1dt;
        coef2[l - 1] = bc;
        hipchk(c, hipMemcpyAsync(c->b, W[l - 1], n * 8, hipMemcpyDeviceToDevice, c->stream), "copy");
        hipchk(c, blas_gemv_add(c->R1all, 0, n, s, coef1, c->b, 0, n, c->stream), "b");
        hipchk(c, blas_gemv_add(c->R2all, 0, n, s, coef2, c->b, 0, n, c->stream), "b");
        pc_use_slot(c, across ? s - 1 + (l - 1) : 0);   // across steps: slots after the correctors'
        newton_solve(c, c->b, a1dt, bc, W[l - 1], W[l], across);
        op_r1r2(c, W[l], R1(l), R2(l));
    }
    // corrector sweeps: every stage of sweep k uses iterate [k] of all stages
    const bool paired = c->prm.pc_rebuild == HBPC_PC_PAIRED;
    for (int k = 0; k < c->prm.kmax; ++k) {
        PhaseRange sweep("corrector sweep");
        for (int l = 1; l < s; ++l) {
            double coef1[4], coef2[4];
            for (int j = 0; j < s; ++j) {
                coef1[j] = dt * t.B1[l][j] - (j == l ? dt : 0.0);
                coef2[j] = dt * dt * t.B2[l][j] + (j == l ? dt * dt / 2 : 0.0);
            }
            if (paired && l + 1 < s) {
                // stages l and l + 1 side by side, on the blocks of slot l - 1 (built at stage l's
                // state in the first sweep, kept for the later ones)
                pair_alloc(c);
                double* bb[2] = {c->b, c->pair.b};
                for (int i = 0; i < 2; ++i) {
                    double cf1[4], cf2[4];
                    for (int j = 0; j < s; ++j) {
                        cf1[j] = dt * t.B1[l + i][j] - (j == l + i ? dt : 0.0);
                        cf2[j] = dt * dt * t.B2[l + i][j] + (j == l + i ? dt * dt / 2 : 0.0);
                    }
                    hipchk(c, hipMemcpyAsync(bb[i], W[0], n * 8, hipMemcpyDeviceToDevice, c->stream), "copy");
                    hipchk(c, blas_gemv_add(c->R1all, 0, n, s, cf1, bb[i], 0, n, c->stream), "b");
                    hipchk(c, blas_gemv_add(c->R2all, 0, n, s, cf2, bb[i], 0, n, c->stream), "b");
                }
                pc_use_slot(c, l - 1);
                const double* gs[2] = {W[l], W[l + 1]};
                double* os[2] = {c->Wn[l], c->Wn[l + 1]};
                newton_solve_pair(c, bb, dt, dt * dt / 2, gs, os, k > 0);
                ++l;
                continue;
            }
            hipchk(c, hipMemcpyAsync(c->b, W[0], n * 8, hipMemcpyDeviceToDevice, c->stream), "copy");
            hipchk(c, blas_gemv_add(c->R1all, 0, n, s, coef1, c->b, 0, n, c->stream), "b");
            hipchk(c, blas_gemv_add(c->R2all, 0, n, s, coef2, c->b, 0, n, c->stream), "b");
            const bool per_stage = c->prm.pc_rebuild == HBPC_PC_PER_STAGE || paired;
            pc_use_slot(c, per_stage || across ? l - 1 : 0);
            newton_solve(c, c->b, dt, dt * dt / 2, W[l], c->Wn[l], (per_stage && k > 0) || across);
        }
        for (int l = 1; l < s; ++l) std::swap(W[l], c->Wn[l]);
        if (k < c->prm.kmax - 1)
            for (int l = 1; l < s; ++l) op_r1r2(c, W[l], R1(l), R2(l));
    }
    status_reset(c);
    hipchk(c, blas_nonfinite(W[s - 1], 0, n, c->dstatus, c->stream), "check");
    if (status_read(c)) set_err(c, HBPC_ERR_NONFINITE, "non-finite value in the new state");
    hipchk(c, hipMemcpyAsync(w_inout, W[s - 1], n * 8, hipMemcpyDeviceToDevice, c->stream), "copy");
    hipchk(c, hipStreamSynchronize(c->stream), "sync");
    pc_use_slot(c, 0);
    if (across) c->pc_steps++;
}

// ------------------------------------------------------------------ context
static void ctx_free(hbpc_ctx* c) {
    for (int i = 0; i < 4; ++i) {
        dfree(c->W[i]);
        dfree(c->Wn[i]);
        dfree(c->tmp[i]);
    }
    void* bufs[] = {c->R1all, c->R2all, c->X, c->b, c->G, c->dX, c->rhs, c->trw, c->trs, c->trd1,
                    c->X32, c->trw32, c->trs32, c->trd1_32, c->V, c->Z, c->kv, c->KT, c->HT,
                    c->part, c->dres, c->dgram, c->dcount, c->dstatus, c->basis64, c->basis32, c->theta, c->adam_m, c->adam_v,
                    c->mgrad, c->theta16, c->gemm_ws, c->ap_X, c->ap_G1, c->ap_G2, c->ap_H1, c->ap_H2, c->ap_Y, c->ap_s, c->tr_buf, c->tr_idx_dev,
                    c->col_elems};
    for (void* p : bufs) dfree(p);
    pair_free(c);
    for (int i = 0; i < 4; ++i) dfree(c->Sinv_slot[i]);
    c->Sinv = nullptr;
    for (int i = 0; i < 6; ++i) dfree(c->fd[i]);
    for (int j = 0; j < 4; ++j) {
        dfree(c->qtr[0][j]);
        dfree(c->qtr[1][j]);
        dfree(c->nsg[0][j]);
        dfree(c->nsg[1][j]);
    }
    if (c->hres) (void)hipHostFree(c->hres);
    for (int i = 0; i < 2; ++i)
        if (c->arn_ev[i]) (void)hipEventDestroy(c->arn_ev[i]);
    for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
    c->ev.clear();
}

// Mesh, degree, equation and flux checks and the geometry of the operator kernels (device
// pointers of the 1-D operators left null); shared by hbpc_create and the context-free R1 entry.
int geom_configure(const hbpc_mesh* mesh, int N, int equation, const hbpc_params* prm, Basis1DHost& basis,
                   GeomHost& g, FamilyLauncher& launch, int& visc, int& ns, std::string& msg) {
    const int D = mesh->dim;
    visc = 0;
    ns = 0;
    if (D < 1 || D > 3) { msg = "dim must be 1, 2 or 3"; return HBPC_ERR_ARG; }
    if (N < 2 || N > 7) { msg = "N must be in 2..7"; return HBPC_ERR_UNSUPPORTED; }
    if (D == 3 && N > 5) { msg = "N must be in 2..5 in 3-D"; return HBPC_ERR_UNSUPPORTED; }
    for (int m = 0; m < D; ++m)
        if (mesh->nelem[m] < 1 || !(mesh->length[m] > 0)) { msg = "bad mesh extent"; return HBPC_ERR_ARG; }
    int NV = 1;
    if (equation == HBPC_EQ_ADVECTION) {
        launch = dg_launch_advection;
    } else if (equation == HBPC_EQ_EULER) {
        if (D < 2) { msg = "Euler needs dim 2 or 3"; return HBPC_ERR_UNSUPPORTED; }
        NV = D + 2;
        launch = dg_launch_euler;
    } else if (equation == HBPC_EQ_NAVIER_STOKES) {
        if (D < 2) { msg = "Navier-Stokes needs dim 2 or 3"; return HBPC_ERR_UNSUPPORTED; }
        if (D == 3 && N > 4) { msg = "Navier-Stokes in 3-D is compiled for N <= 4"; return HBPC_ERR_UNSUPPORTED; }
        NV = D + 2;
        ns = 1;
        launch = dg_launch_ns;
    } else if (equation == HBPC_EQ_BURGERS_BR1) {
        if (D > 2) { msg = "viscous Burgers is compiled for dim 1 and 2"; return HBPC_ERR_UNSUPPORTED; }
        visc = 1;
        launch = dg_launch_burgers;
    } else {
        msg = "unknown equation";
        return HBPC_ERR_ARG;
    }
    if (prm->flux < 0 || prm->flux > 4) { msg = "unknown flux"; return HBPC_ERR_ARG; }
    const bool euler_like = equation == HBPC_EQ_EULER || equation == HBPC_EQ_NAVIER_STOKES;
    if ((prm->flux == HBPC_FLUX_RUSANOV || prm->flux == HBPC_FLUX_LF_LITERAL) && !euler_like) {
        msg = "Rusanov and lf_literal fluxes need the Euler or Navier-Stokes equations";
        return HBPC_ERR_ARG;
    }
    if (prm->flux == HBPC_FLUX_UPWIND && equation != HBPC_EQ_ADVECTION) {
        msg = "upwind flux needs advection";
        return HBPC_ERR_ARG;
    }
    if (equation == HBPC_EQ_BURGERS_BR1 && !(prm->nu >= 0)) { msg = "nu must be >= 0"; return HBPC_ERR_ARG; }
    if (euler_like && !(prm->eps_ref > 0 && prm->gamma > 1)) {
        msg = "Euler needs gamma > 1 and eps_ref > 0";
        return HBPC_ERR_ARG;
    }
    if (ns && !(prm->mu >= 0 && prm->prandtl > 0 && prm->eta_br2 >= 0)) {
        msg = "Navier-Stokes needs mu >= 0, prandtl > 0 and eta_br2 >= 0";
        return HBPC_ERR_ARG;
    }
    if (!basis1d_build(N, prm->nodes, basis)) { msg = "bad node set"; return HBPC_ERR_ARG; }
    std::memset(&g, 0, sizeof(g));
    g.D = D;
    g.NP = N + 1;
    g.NV = NV;
    g.nE = 1;
    for (int m = 0; m < D; ++m) g.nE *= mesh->nelem[m];
    for (int m = 0; m < 3; ++m) {
        g.nel[m] = m < D ? mesh->nelem[m] : 1;
        g.two_h[m] = m < D ? 2.0 * mesh->nelem[m] / mesh->length[m] : 0.0;
        g.adv[m] = prm->adv[m];
    }
    g.lam = prm->lambda;
    g.nu = prm->nu;
    g.gamma = euler_like ? prm->gamma : 1.4;
    g.eps = euler_like ? prm->eps_ref : 1.0;
    if (ns) {
        const double R = 1.0 / (g.gamma * g.eps * g.eps);
        g.mu = prm->mu;
        g.kappa = R * g.gamma / (g.gamma - 1.0) * prm->mu / prm->prandtl;
        g.gam_eps2 = 1.0 / R;
        g.eta = prm->eta_br2;
    }
    g.flux = prm->flux;
    return HBPC_OK;
}

// 1-D operators in the kernels' layout: Dhat, l(+1), l(-1), lhat(+1), lhat(-1), and for BR2 the
// strong derivative, its interpolant's values at +-1 and c_+-
std::vector<double> basis_table(const Basis1DHost& b) {
    std::vector<double> hb;
    hb.insert(hb.end(), b.Dhat.begin(), b.Dhat.end());
    hb.insert(hb.end(), b.lp.begin(), b.lp.end());
    hb.insert(hb.end(), b.lm.begin(), b.lm.end());
    hb.insert(hb.end(), b.lhp.begin(), b.lhp.end());
    hb.insert(hb.end(), b.lhm.begin(), b.lhm.end());
    hb.insert(hb.end(), b.Dstr.begin(), b.Dstr.end());
    hb.insert(hb.end(), b.lDp.begin(), b.lDp.end());
    hb.insert(hb.end(), b.lDm.begin(), b.lDm.end());
    hb.push_back(b.cp);
    hb.push_back(b.cm);
    return hb;
}

static void ctx_init(hbpc_ctx* c, const hbpc_mesh* mesh, int N, int equation, const hbpc_params* prm) {
    const char* vb = std::getenv("HBPC_VERBOSE");
    c->verbose = vb && vb[0] && vb[0] != '0';
    c->prof_only = -1;
    c->mesh = *mesh;
    c->prm = *prm;
    c->N = N;
    c->NP = N + 1;
    c->D = mesh->dim;
    c->equation = equation;
    {
        std::string msg;
        const int rc = geom_configure(mesh, N, equation, prm, c->basis, c->geom, c->launch, c->visc, c->ns, msg);
        if (rc != HBPC_OK) set_err(c, rc, msg);
    }
    c->NV = c->geom.NV;
    if (prm->gmres_restart < 1 || prm->gmres_restart > HBPC_MAX_RESTART)
        set_err(c, HBPC_ERR_ARG, "gmres_restart must be 1.." + std::to_string(HBPC_MAX_RESTART));
    if (prm->precond < HBPC_PC_NONE || prm->precond > HBPC_PC_BJEXT_H)
        set_err(c, HBPC_ERR_ARG, "unknown precond");
    if (prm->pc_rebuild < HBPC_PC_PER_SOLVE || prm->pc_rebuild > HBPC_PC_PAIRED)
        set_err(c, HBPC_ERR_ARG, "unknown pc_rebuild");
    if (prm->pc_rebuild == HBPC_PC_PAIRED && ((prm->precond != HBPC_PC_BJEXT && prm->precond != HBPC_PC_LEARNED) ||
                                              prm->jvp_mode != HBPC_JVP_LINEARISED))
        set_err(c, HBPC_ERR_ARG, "HBPC_PC_PAIRED needs BJ_ext or the learned preconditioner and the linearised JVP");
    if (prm->pc_rebuild == HBPC_PC_ACROSS_STEPS && prm->q > 6)
        set_err(c, HBPC_ERR_ARG, "HBPC_PC_ACROSS_STEPS keeps 2 (s - 1) block sets: q <= 6");
    if (prm->pc_rebuild == HBPC_PC_ACROSS_STEPS && prm->pc_reuse_steps < 1)
        set_err(c, HBPC_ERR_ARG, "pc_reuse_steps must be >= 1");
    if (prm->pc_probe_its < 0) set_err(c, HBPC_ERR_ARG, "pc_probe_its must be >= 0");
    if (prm->mlp_precision != HBPC_MLP_BF16 && prm->mlp_precision != HBPC_MLP_FP32)
        set_err(c, HBPC_ERR_ARG, "unknown mlp_precision");
    if (prm->q != 4 && prm->q != 6 && prm->q != 8) set_err(c, HBPC_ERR_ARG, "q must be 4, 6 or 8");
    if (prm->kmax < 0) set_err(c, HBPC_ERR_ARG, "kmax must be >= 0");
    c->stream = (hipStream_t)prm->stream;
    c->NN = 1;
    c->NFP = 1;
    for (int m = 0; m < c->D; ++m) c->NN *= c->NP;
    for (int m = 0; m + 1 < c->D; ++m) c->NFP *= c->NP;
    c->NE = c->NV * c->NN;
    c->nE = c->geom.nE;
    c->ndof = (size_t)c->nE * c->NE;
    c->n2 = 2 * c->ndof;
    c->tsz = (size_t)c->nE * 2 * c->D * c->NV * c->NFP;
    GeomHost& g = c->geom;

    const size_t n = c->ndof;
    {   // 1-D operators
        std::vector<double> hb = basis_table(c->basis);
        std::vector<float> hf(hb.begin(), hb.end());
        c->basis64 = dalloc<double>(c, hb.size());
        c->basis32 = dalloc<float>(c, hf.size());
        hipchk(c, hipMemcpy(c->basis64, hb.data(), hb.size() * 8, hipMemcpyHostToDevice), "copy basis");
        hipchk(c, hipMemcpy(c->basis32, hf.data(), hf.size() * 4, hipMemcpyHostToDevice), "copy basis");
        g.basis64 = c->basis64;
        g.basis32 = c->basis32;
    }
    for (int i = 0; i < 4; ++i) {
        c->W[i] = dalloc<double>(c, n);
        c->Wn[i] = dalloc<double>(c, n);
        c->tmp[i] = dalloc<double>(c, n);
    }
    c->R1all = dalloc<double>(c, 4 * n);
    c->R2all = dalloc<double>(c, 4 * n);
    c->X = dalloc<double>(c, 2 * n);
    c->b = dalloc<double>(c, n);
    c->G = dalloc<double>(c, 2 * n);
    c->dX = dalloc<double>(c, 2 * n);
    c->rhs = dalloc<double>(c, 2 * n);
    c->trw = dalloc<double>(c, c->tsz);
    c->trs = dalloc<double>(c, c->tsz);
    c->trd1 = dalloc<double>(c, 2 * c->tsz);   // trd2 follows trd1 (one trace launch for dX)
    c->trd2 = c->trd1 + c->tsz;
    c->X32 = dalloc<float>(c, 2 * n);
    c->trw32 = dalloc<float>(c, c->tsz);
    c->trs32 = dalloc<float>(c, c->tsz);
    c->trd1_32 = dalloc<float>(c, 2 * c->tsz);
    c->trd2_32 = c->trd1_32 + c->tsz;
    if (c->visc)
        for (int j = 0; j < 4; ++j) {
            c->qtr[0][j] = dalloc<double>(c, c->tsz);
            c->qtr[1][j] = dalloc<float>(c, c->tsz);
        }
    if (c->ns) {   // per element, face and face point: the nvar components of the viscous flux
        const size_t gsz = (size_t)c->nE * 2 * c->D * c->NV * c->NFP;
        for (int j = 0; j < 4; ++j) {
            c->nsg[0][j] = dalloc<double>(c, gsz);
            c->nsg[1][j] = dalloc<float>(c, gsz);
        }
    }
    c->m_alloc = prm->gmres_restart;
    c->kr_f32 = prm->precision == HBPC_MIXED;
    size_t ksz = c->kr_f32 ? 4 : 8;
    c->V = dalloc<char>(c, (size_t)(c->m_alloc + 1) * c->n2 * ksz);
    c->Z = prm->precond != HBPC_PC_NONE ? (void*)dalloc<char>(c, (size_t)c->m_alloc * c->n2 * ksz) : nullptr;
    // learned preconditioner: network shape and FP32 parameters / Adam moments / gradient
    c->mlp_H = 256;
    c->mlp_nin = (2 * c->D + 1) * 2 * c->NE + 2;
    c->mlp_nr = (2 * c->D + 1) * c->NE;
    {
        const size_t nr = c->mlp_nr, nw = c->mlp_nin - c->mlp_nr, H = c->mlp_H, no = c->NE;
        c->mlp_np = nr * H + nw * H + H + 2 * H * H + H + H * no;
    }
    c->theta = dalloc<float>(c, c->mlp_np);
    c->adam_m = dalloc<float>(c, c->mlp_np);
    c->adam_v = dalloc<float>(c, c->mlp_np);
    c->mgrad = dalloc<float>(c, c->mlp_np);
    c->theta16 = dalloc<uint16_t>(c, c->mlp_np);
    c->gemm_ws_floats = (size_t)4 << 20;   // 16 MiB: 512 + 256 output tiles of 64 x 64 (see mlp_gemm)
    c->gemm_ws = dalloc<float>(c, c->gemm_ws_floats);
    c->lpc_snap = -1;
    c->kv = dalloc<double>(c, 3 * n);
    // K build in chunks of <= 4 GiB of FP64 blocks (the whole 128^2 N=5 mesh in one launch, so the
    // inversion kernel runs tens of workgroup rounds instead of three with a 16 % tail)
    size_t per = (size_t)c->NE * c->NE * 8;
    c->kt_chunk = std::max<size_t>(1, std::min<size_t>(c->nE, ((size_t)4 << 30) / per));
    // block partials of up to 2 (m + 1) columns; device results: one Arnoldi slot (h1 | g of
    // 2 (m + 1), ||u||^2 in 4, h of m + 1), then the norm and loss words
    c->part = dalloc<double>(c, (size_t)blas_mdot_grid(c->n2) * (2 * (c->m_alloc + 1) + 2) + 64);
    c->arn_len = 3 * ((size_t)c->m_alloc + 1) + 8;
    c->dres = dalloc<double>(c, c->arn_len + 64);
    c->dgram = dalloc<double>(c, (size_t)(c->m_alloc + 1) * (c->m_alloc + 1));
    c->dcount = dalloc<unsigned>(c, 4);
    hipchk(c, hipMemset(c->dcount, 0, 4 * sizeof(unsigned)), "memset");
    c->dstatus = dalloc<int>(c, 1);
    void* h = nullptr;
    hipchk(c, hipHostMalloc(&h, (2 * c->arn_len + 64) * sizeof(double)), "hipHostMalloc");
    c->hres = (double*)h;
    for (int i = 0; i < 2; ++i) hipchk(c, hipEventCreateWithFlags(&c->arn_ev[i], hipEventDisableTiming), "event");
}

static void train_impl(hbpc_ctx* c, const float* X, const float* T, size_t count, const hbpc_train_cfg* cfg,
                       hbpc_train_log* log) {
    const double t0 = now_ms();
    if (!c->mlp_ready) set_err(c, HBPC_ERR_ARG, "hbpc_mlp_set_params before training");
    const int B = (int)std::min<size_t>((size_t)cfg->batch, count);
    const int ni = c->mlp_nin, no = c->NE, bf16 = cfg->precision == HBPC_MLP_BF16;
    mlp_train_alloc(c, B);
    if (c->tr_idx_cap < count) {
        dfree(c->tr_idx_dev);
        c->tr_idx_dev = nullptr;
        c->tr_idx_cap = 0;
        c->tr_idx_dev = dalloc<int>(c, count);
        c->tr_idx_cap = count;
    }
    // batch buffers behind the activations of mlp_loss_grad_dev
    float* Xb = c->tr_buf + (size_t)B * (10 * (size_t)c->mlp_H + 2 * (size_t)no);
    float* Tb = Xb + (size_t)B * ni;
    std::vector<int> perm(count);
    unsigned long long state = cfg->seed;
    double* sse = c->dres + c->arn_len + 8;
    int steps = 0;
    double first = 0.0, last = 0.0;
    for (int ep = 0; ep < cfg->epochs; ++ep) {
        for (size_t i = 0; i < count; ++i) perm[i] = (int)i;
        for (size_t i = count - 1; i > 0; --i) {
            size_t j = (size_t)(splitmix64(state) % (unsigned long long)(i + 1));
            std::swap(perm[i], perm[j]);
        }
        hipchk(c, hipMemcpyAsync(c->tr_idx_dev, perm.data(), count * sizeof(int), hipMemcpyHostToDevice,
                                 c->stream),
               "copy");
        hipchk(c, hipMemsetAsync(sse, 0, sizeof(double), c->stream), "memset");
        for (size_t b0 = 0; b0 < count; b0 += B) {
            const int rows = (int)std::min<size_t>(B, count - b0);
            hipchk(c, mlp_gather(X, ni, c->tr_idx_dev + b0, rows, ni, Xb, c->stream), "gather");
            hipchk(c, mlp_gather(T, no, c->tr_idx_dev + b0, rows, no, Tb, c->stream), "gather");
            mlp_loss_grad_dev(c, Xb, Tb, rows, c->mgrad, sse, bf16);
            mlp_adam_dev(c, c->mgrad, cfg->lr, cfg->beta1, cfg->beta2, cfg->eps);
            ++steps;
        }
        double h = 0.0;
        hipchk(c, hipMemcpyAsync(&h, sse, sizeof(double), hipMemcpyDeviceToHost, c->stream), "copy");
        hipchk(c, hipStreamSynchronize(c->stream), "sync");   // perm is reused by the next epoch
        const double mean = h / ((double)count * no);
        if (!std::isfinite(mean)) set_err(c, HBPC_ERR_NONFINITE, "non-finite training loss");
        if (ep == 0) first = mean;
        last = mean;
    }
    if (log) {
        log->steps = steps;
        log->loss_first = first;
        log->loss_last = last;
        log->ms = now_ms() - t0;
    }
}

static void mlp_init_impl(hbpc_ctx* c, unsigned long long seed) {
    float* b[7];
    mlp_blocks(c, c->theta, b);
    const long long nr = c->mlp_nr, nw = c->mlp_nin - c->mlp_nr, H = c->mlp_H, no = c->NE;
    const long long rows[7] = {nr, nw, 0, H, H, 0, H}, cols[7] = {H, H, H, H, H, H, no};
    for (int k = 0; k < 7; ++k) {
        if (rows[k] == 0) {   // biases
            hipchk(c, hipMemsetAsync(b[k], 0, cols[k] * sizeof(float), c->stream), "memset");
            continue;
        }
        const double gain = (k == 1 || k == 4) ? 6.0 : 3.0;   // W1w, W2w feed a ReLU
        hipchk(c, mlp_uniform(b[k], rows[k] * cols[k], (float)std::sqrt(gain / (double)rows[k]),
                              seed ^ (0x632BE59BD9B4E019ull * (unsigned long long)(k + 1)), c->stream),
               "init");
    }
    const size_t bytes = c->mlp_np * sizeof(float);
    hipchk(c, hipMemsetAsync(c->adam_m, 0, bytes, c->stream), "memset");
    hipchk(c, hipMemsetAsync(c->adam_v, 0, bytes, c->stream), "memset");
    hipchk(c, mlp_to_bf16(c->theta, c->theta16, (long long)c->mlp_np, c->stream), "bf16 copy");
    c->adam_t = 0;
    c->mlp_ready = 1;
}

// ------------------------------------------------------------------ C ABI
#define HBPC_TRY(ctx, body)                              \
    try {                                                \
        body;                                            \
        return HBPC_OK;                                  \
    } catch (const Fail& f) {                            \
        return f.code;                                   \
    } catch (...) {                                      \
        if (ctx) (ctx)->err = "unexpected C++ exception"; \
        return HBPC_ERR_ARG;                             \
    }

extern "C" {

void hbpc_default_params(hbpc_params* p) {
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->nodes = HBPC_NODES_GAUSS;
    p->flux = HBPC_FLUX_RUSANOV;
    p->lambda = 1.0;
    p->adv[0] = 1.0;
    p->nu = 0.0;
    p->gamma = 1.4;
    p->eps_ref = 1.0;
    p->mu = 0.0;
    p->prandtl = 0.72;
    p->eta_br2 = 2.0;
    p->q = 6;
    p->kmax = 4;
    p->newton_rtol = 1e-8;
    p->newton_atol_dw = 1.95e-15;   // 1e-12 in the 2-norm over 262,144 coefficients
    p->newton_maxit = 30;
    p->gmres_rtol = 1e-3;
    p->gmres_restart = 30;
    p->gmres_maxit = 7000;
    p->precision = HBPC_FP64;
    p->precond = HBPC_PC_BJEXT;
    p->pc_rebuild = HBPC_PC_PER_SOLVE;
    p->jvp_mode = HBPC_JVP_LINEARISED;
    p->hessian = 1;
    p->mlp_precision = HBPC_MLP_BF16;
    p->pc_fallback = 0.5;
    p->pc_reuse_steps = 4;
    p->pc_probe_its = 0;
    p->stream = nullptr;
}

int hbpc_create(const hbpc_mesh* mesh, int N, int equation, const hbpc_params* params, hbpc_ctx** out) {
    if (!mesh || !params || !out) return HBPC_ERR_ARG;
    *out = nullptr;
    hbpc_ctx* c = new (std::nothrow) hbpc_ctx();
    if (!c) return HBPC_ERR_OOM;
    try {
        ctx_init(c, mesh, N, equation, params);
    } catch (const Fail& f) {
        ctx_free(c);
        delete c;
        return f.code;
    }
    *out = c;
    return HBPC_OK;
}

int hbpc_destroy(hbpc_ctx* c) {
    if (!c) return HBPC_ERR_ARG;
    (void)hipStreamSynchronize(c->stream);
    ctx_free(c);
    delete c;
    return HBPC_OK;
}

int hbpc_set_stream(hbpc_ctx* c, void* stream) {
    if (!c) return HBPC_ERR_ARG;
    c->stream = (hipStream_t)stream;
    c->prm.stream = stream;
    return HBPC_OK;
}

size_t hbpc_ndof(const hbpc_ctx* c) { return c ? c->ndof : 0; }

int hbpc_block_size(const hbpc_ctx* c) { return c ? c->NE : 0; }

int hbpc_nodes(const hbpc_ctx* c, double* xi, double* w) {
    if (!c || !xi || !w) return HBPC_ERR_ARG;
    for (int i = 0; i < c->NP; ++i) {
        xi[i] = c->basis.xi[i];
        w[i] = c->basis.w[i];
    }
    return HBPC_OK;
}

int hbpc_residual1(hbpc_ctx* c, const double* w, double* r1) {
    if (!c || !w || !r1) return HBPC_ERR_ARG;
    HBPC_TRY(c, op_r1(c, w, r1, c->trw));
}

int hbpc_residual2(hbpc_ctx* c, const double* w, const double* sigma, double* r2) {
    if (!c || !w || !r2) return HBPC_ERR_ARG;
    HBPC_TRY(c, {
        if (!sigma) {
            op_r1(c, w, c->tmp[0], c->trw);
            sigma = c->tmp[0];
        } else {
            op_trace(c, w, c->trw, 0);
        }
        op_trace(c, sigma, c->trs, 0);
        op_r2_tr(c, w, sigma, c->trw, c->trs, r2);
    });
}

int hbpc_newton_residual(hbpc_ctx* c, const double* w, const double* sigma, const double* b, double a1dt,
                         double bcoef, double* G) {
    if (!c || !w || !sigma || !b || !G) return HBPC_ERR_ARG;
    HBPC_TRY(c, {
        op_trace(c, w, c->trw, 0);
        op_trace(c, sigma, c->trs, 0);
        LaunchReq r = op_req(c, OPK_RES);
        r.fld[0] = w;
        r.fld[1] = sigma;
        r.fld[2] = b;
        r.trc[0] = c->trw;
        r.trc[1] = c->trs;
        r.qtr[0] = op_lift(c, w, c->trw, 0, 0);
        r.qtr[1] = op_lift(c, sigma, c->trs, 1, 0);
        r.out[0] = G;
        r.out[1] = G + c->ndof;
        r.c0 = a1dt;
        r.c1 = bcoef;
        op_launch(c, r, 0);
    });
}

int hbpc_jvp(hbpc_ctx* c, const double* w, const double* sigma, double a1dt, double bcoef, const double* dX,
             double* JdX, int mode) {
    if (!c || !w || !sigma || !dX || !JdX) return HBPC_ERR_ARG;
    if (mode != HBPC_JVP_LINEARISED && mode != HBPC_JVP_FD) return HBPC_ERR_ARG;
    HBPC_TRY(c, {
        op_trace(c, w, c->trw, 0);
        op_trace(c, sigma, c->trs, 0);
        if (mode == HBPC_JVP_FD) {
            fd_alloc(c);
            op_r1(c, w, c->fd[0], c->trd1);
            op_r2_tr(c, w, sigma, c->trw, c->trs, c->fd[1]);
            op_jvp_fd(c, w, sigma, dX, JdX, a1dt, bcoef);
        } else {
            op_jvp(c, w, sigma, c->trw, c->trs, dX, JdX, a1dt, bcoef, 0, c->prm.hessian);
        }
    });
}

int hbpc_jvp_f32(hbpc_ctx* c, const float* w, const float* sigma, double a1dt, double bcoef, const float* dX,
                 float* JdX) {
    if (!c || !w || !sigma || !dX || !JdX) return HBPC_ERR_ARG;
    HBPC_TRY(c, {
        op_trace(c, w, c->trw32, 1);
        op_trace(c, sigma, c->trs32, 1);
        op_jvp(c, w, sigma, c->trw32, c->trs32, dX, JdX, a1dt, bcoef, 1, c->prm.hessian);
    });
}

// sigma: nullptr for BJ_ext (or the learned snapshot), the state's sigma for BJ^H_ext
static void pc_build_abi(hbpc_ctx* c, const double* w, const double* sigma, double a1dt, double bcoef,
                         int precision) {
    c->pc_steps = 1 << 30;   // slot 0 is overwritten: blocks kept across steps are rebuilt next step
    const int f32 = precision == HBPC_MIXED;
    const int learned = c->prm.precond == HBPC_PC_LEARNED;
    pc_use_slot(c, 0);
    if (learned && sigma)
        set_err(c, HBPC_ERR_ARG, "hbpc_pc_build_hess on a context with the learned preconditioner");
    if (learned && !c->mlp_ready) set_err(c, HBPC_ERR_ARG, "learned preconditioner without parameters");
    if (!learned) pc_build(c, w, sigma, a1dt, bcoef, f32);
    if (f32) {
        hipchk(c, blas_axpby(1.0, w, 0, 0.0, c->X32, 1, c->ndof, c->stream), "cast");
        op_trace(c, c->X32, c->trw32, 1);
    } else {
        hipchk(c, hipMemcpyAsync(c->tmp[1], w, c->ndof * 8, hipMemcpyDeviceToDevice, c->stream), "copy");
    }
    if (learned) {
        lpc_prepare(c, f32 ? (const void*)c->X32 : (const void*)c->tmp[1], f32, a1dt, bcoef);
        c->lpc_snap = f32;
    }
}

int hbpc_pc_build(hbpc_ctx* c, const double* w, double a1dt, double bcoef, int precision) {
    if (!c || !w) return HBPC_ERR_ARG;
    HBPC_TRY(c, { pc_build_abi(c, w, nullptr, a1dt, bcoef, precision); });
}

int hbpc_pc_build_hess(hbpc_ctx* c, const double* w, const double* sigma, double a1dt, double bcoef, int precision) {
    if (!c || !w || !sigma) return HBPC_ERR_ARG;
    HBPC_TRY(c, { pc_build_abi(c, w, sigma, a1dt, bcoef, precision); });
}

int hbpc_pc_apply(hbpc_ctx* c, const double* X, double* Y) {
    if (!c || !X || !Y) return HBPC_ERR_ARG;
    const int learned = c->prm.precond == HBPC_PC_LEARNED;
    if (learned ? c->lpc_snap != 0 : (!c->pc_valid || c->sinv_f32)) {
        c->err = "hbpc_pc_apply needs an FP64 hbpc_pc_build first";
        return HBPC_ERR_ARG;
    }
    HBPC_TRY(c, {
        op_trace(c, c->tmp[1], c->trw, 0);
        if (learned) lpc_apply(c, c->tmp[1], c->trw, X, Y, 0);
        else pc_apply(c, c->tmp[1], c->trw, X, Y, 0);
    });
}

int hbpc_pc_apply_f32(hbpc_ctx* c, const float* X, float* Y) {
    if (!c || !X || !Y) return HBPC_ERR_ARG;
    const int learned = c->prm.precond == HBPC_PC_LEARNED;
    if (learned ? c->lpc_snap != 1 : (!c->pc_valid || !c->sinv_f32)) {
        c->err = "hbpc_pc_apply_f32 needs an HBPC_MIXED hbpc_pc_build first";
        return HBPC_ERR_ARG;
    }
    HBPC_TRY(c, {
        if (learned) lpc_apply(c, c->X32, c->trw32, X, Y, 1);
        else pc_apply(c, c->X32, c->trw32, X, Y, 1);
    });
}

// ---- learned preconditioner network
int hbpc_mlp_shape(const hbpc_ctx* c, int* n_in, int* hidden, int* n_out, size_t* n_params) {
    if (!c) return HBPC_ERR_ARG;
    if (n_in) *n_in = c->mlp_nin;
    if (hidden) *hidden = c->mlp_H;
    if (n_out) *n_out = c->NE;
    if (n_params) *n_params = c->mlp_np;
    return HBPC_OK;
}

int hbpc_mlp_set_params(hbpc_ctx* c, const float* theta) {
    if (!c || !theta) return HBPC_ERR_ARG;
    HBPC_TRY(c, {
        const size_t b = c->mlp_np * sizeof(float);
        hipchk(c, hipMemcpyAsync(c->theta, theta, b, hipMemcpyDeviceToDevice, c->stream), "copy");
        hipchk(c, mlp_to_bf16(c->theta, c->theta16, (long long)c->mlp_np, c->stream), "bf16 copy");
        hipchk(c, hipMemsetAsync(c->adam_m, 0, b, c->stream), "memset");
        hipchk(c, hipMemsetAsync(c->adam_v, 0, b, c->stream), "memset");
        c->adam_t = 0;
        c->mlp_ready = 1;
    });
}

int hbpc_mlp_init(hbpc_ctx* c, unsigned long long seed) {
    if (!c) return HBPC_ERR_ARG;
    HBPC_TRY(c, mlp_init_impl(c, seed));
}

int hbpc_mlp_get_params(hbpc_ctx* c, float* theta) {
    if (!c || !theta) return HBPC_ERR_ARG;
    HBPC_TRY(c, hipchk(c, hipMemcpyAsync(theta, c->theta, c->mlp_np * sizeof(float), hipMemcpyDeviceToDevice,
                                         c->stream),
                       "copy"));
}

int hbpc_mlp_features(hbpc_ctx* c, const double* rt, const double* w, const double* dw, const int* elems, int count,
                      double a1dt, double bcoef, float* X, float* T, float* scale) {
    if (!c || !rt || !w || !X || count < 0 || (dw && !T)) return HBPC_ERR_ARG;
    if (!elems && count > c->nE) return HBPC_ERR_ARG;
    HBPC_TRY(c, features_p(c, rt, w, dw, 0, elems, count, a1dt, bcoef, X, dw ? T : nullptr, scale, 3));
}

int hbpc_mlp_forward(hbpc_ctx* c, const float* X, int rows, float* Y, int precision) {
    if (!c || !X || !Y || rows < 0) return HBPC_ERR_ARG;
    if (precision != HBPC_MLP_BF16 && precision != HBPC_MLP_FP32) return HBPC_ERR_ARG;
    HBPC_TRY(c, {
        mlp_train_alloc(c, rows);
        const size_t RH = (size_t)rows * c->mlp_H;
        float* G1 = c->tr_buf;
        const int bf16 = precision == HBPC_MLP_BF16;
        mlp_gates(c, X, rows, G1, G1 + RH, bf16);
        mlp_residual_path(c, X, rows, G1, G1 + RH, G1 + 2 * RH, G1 + 3 * RH, Y, bf16);
    });
}

int hbpc_mlp_loss_grad(hbpc_ctx* c, const float* X, const float* T, int rows, float* grad, double* loss_host,
                       int precision) {
    if (!c || !X || !T || !grad || rows <= 0) return HBPC_ERR_ARG;
    if (precision != HBPC_MLP_BF16 && precision != HBPC_MLP_FP32) return HBPC_ERR_ARG;
    HBPC_TRY(c, {
        double* sse = c->dres + c->arn_len + 8;
        hipchk(c, hipMemsetAsync(sse, 0, sizeof(double), c->stream), "memset");
        mlp_loss_grad_dev(c, X, T, rows, grad, sse, precision == HBPC_MLP_BF16);
        double h = 0.0;
        hipchk(c, hipMemcpyAsync(&h, sse, sizeof(double), hipMemcpyDeviceToHost, c->stream), "copy");
        hipchk(c, hipStreamSynchronize(c->stream), "sync");
        if (loss_host) *loss_host = h / ((double)rows * c->NE);
    });
}

int hbpc_mlp_adam(hbpc_ctx* c, const float* grad, double lr, double beta1, double beta2, double eps) {
    if (!c || !grad) return HBPC_ERR_ARG;
    HBPC_TRY(c, mlp_adam_dev(c, grad, lr, beta1, beta2, eps));
}

int hbpc_mlp_collect(hbpc_ctx* c, float* X, float* T, size_t capacity, int per_event, unsigned long long seed,
                     int source, int every) {
    if (!c) return HBPC_ERR_ARG;
    if (capacity == 0) {
        c->col_X = c->col_T = nullptr;
        c->col_cap = 0;
        return HBPC_OK;
    }
    if (!X || !T || per_event < 1 || every < 1) return HBPC_ERR_ARG;
    if (source < HBPC_MLP_PAIRS_NEWTON || source > HBPC_MLP_PAIRS_RANDOM) return HBPC_ERR_ARG;
    c->col_source = source;
    c->col_every = every;
    HBPC_TRY(c, {
        if (!c->col_elems) c->col_elems = dalloc<int>(c, c->nE);
        c->col_X = X;
        c->col_T = T;
        c->col_cap = capacity;
        c->col_count = 0;
        c->col_per = per_event;
        c->col_seed = seed;
        c->col_draws = 0;
    });
}

size_t hbpc_mlp_collected(const hbpc_ctx* c) { return c ? c->col_count : 0; }

void hbpc_default_train_cfg(hbpc_train_cfg* cfg) {
    if (!cfg) return;
    std::memset(cfg, 0, sizeof(*cfg));
    cfg->epochs = 40;
    cfg->batch = 256;
    cfg->lr = 1e-3;
    cfg->beta1 = 0.9;
    cfg->beta2 = 0.999;
    cfg->eps = 1e-8;
    cfg->seed = 2109;
    cfg->precision = HBPC_MLP_BF16;
}

int hbpc_train_mlp(hbpc_ctx* c, const float* X, const float* T, size_t count, const hbpc_train_cfg* cfg,
                   hbpc_train_log* log) {
    if (!c || !X || !T || !cfg || count == 0) return HBPC_ERR_ARG;
    if (cfg->epochs < 1 || cfg->batch < 1 || cfg->batch > 8192 || !(cfg->lr > 0)) return HBPC_ERR_ARG;
    if (cfg->precision != HBPC_MLP_BF16 && cfg->precision != HBPC_MLP_FP32) return HBPC_ERR_ARG;
    if (count > (size_t)0x7fffffff) return HBPC_ERR_ARG;
    HBPC_TRY(c, train_impl(c, X, T, count, cfg, log));
}

int hbpc_step(hbpc_ctx* c, double* w_inout, double dt, hbpc_stats* stats) {
    if (!c || !w_inout || !(dt > 0)) return HBPC_ERR_ARG;
    if ((c->prm.precision == HBPC_MIXED) != (c->kr_f32 == 1)) {
        c->err = "precision differs from the one the context was created with";
        return HBPC_ERR_ARG;
    }
    std::memset(&c->st, 0, sizeof(c->st));
    c->cur_solve = 0;
    double t0 = now_ms();
    int rc = HBPC_OK;
    try {
        hbpc_step_impl(c, w_inout, dt);
    } catch (const Fail& f) {
        rc = f.code;
        (void)hipStreamSynchronize(c->stream);
    } catch (...) {
        c->err = "unexpected C++ exception";
        rc = HBPC_ERR_ARG;
    }
    c->st.t_step_ms = now_ms() - t0;
    if (stats) *stats = c->st;
    prof_resolve(c);
    return rc;
}

int hbpc_profile_enable(hbpc_ctx* c, int enable) {
    if (!c) return HBPC_ERR_ARG;
    c->prof = enable ? 1 : 0;
    c->prof_only = -1;
    return HBPC_OK;
}

int hbpc_profile_only(hbpc_ctx* c, const char* name) {
    if (!c) return HBPC_ERR_ARG;
    if (!name) {
        c->prof_only = -1;
        return HBPC_OK;
    }
    for (int i = 0; i < KC_COUNT; ++i)
        if (std::strcmp(name, KC_NAMES[i]) == 0) {
            c->prof_only = i;
            return HBPC_OK;
        }
    c->err = std::string("unknown kernel class ") + name;
    return HBPC_ERR_ARG;
}

int hbpc_profile_read(hbpc_ctx* c, hbpc_kernel_prof* out, int max, int reset) {
    if (!c || (max > 0 && !out)) return HBPC_ERR_ARG;
    prof_resolve(c);
    int k = 0;
    for (int i = 0; i < KC_COUNT && k < max; ++i) {
        if (c->kp_launch[i] == 0) continue;
        std::memset(&out[k], 0, sizeof(out[k]));
        std::strncpy(out[k].name, KC_NAMES[i], sizeof(out[k].name) - 1);
        out[k].launches = c->kp_launch[i];
        out[k].total_ms = c->kp_ms[i];
        out[k].bytes = c->kp_bytes[i];
        out[k].flops = c->kp_flops[i];
        ++k;
    }
    if (reset) {
        for (int i = 0; i < KC_MAXCLS; ++i) {
            c->kp_launch[i] = 0;
            c->kp_ms[i] = c->kp_bytes[i] = c->kp_flops[i] = 0.0;
        }
    }
    return k;
}

const char* hbpc_strerror(int code) {
    switch (code) {
    case HBPC_OK: return "ok";
    case HBPC_ERR_ARG: return "invalid argument";
    case HBPC_ERR_OOM: return "out of device memory";
    case HBPC_ERR_HIP: return "HIP runtime error";
    case HBPC_ERR_NONFINITE: return "non-finite value";
    case HBPC_ERR_NEWTON: return "Newton did not converge";
    case HBPC_ERR_GMRES: return "GMRES did not converge";
    case HBPC_ERR_UNSUPPORTED: return "unsupported configuration";
    default: return "unknown error";
    }
}

const char* hbpc_last_error(const hbpc_ctx* c) { return c ? c->err.c_str() : "null context"; }

}  // extern "C"
